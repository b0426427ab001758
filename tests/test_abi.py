"""The C ABI library loads and exports every function include/treebbox.h
declares; host-side argument checks return their status codes before any
device work (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "treebbox.h")
LIB = os.path.join(ROOT, "paper_2205_11659_amd", "libtreebbox.so")

TB_OK, TB_ERR_NULL, TB_ERR_SIZE, TB_ERR_ALIGN, TB_ERR_WORKSPACE, TB_ERR_ARG, TB_ERR_HIP = range(7)


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2205_11659_amd import _build
        _build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    fns = declared_functions()
    for f in ("tb_match", "tb_bbox", "tb_bbox_backward", "tb_bbox_batched", "tb_compose",
              "tb_bbox_stream", "tb_compose_f32", "tb_match_brackets", "tb_bbox_noalloc",
              "tb_tune_bbox", "tb_variant_get",
              "tb_workspace_bytes", "tb_status_str"):
        assert f in fns


def test_every_declared_symbol_is_exported(lib):
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_workspace_bytes(lib):
    f = lib.tb_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64]
    for op in (0, 1, 2, 3, 4, 5, 6, 7):
        assert f(op, 0, 1) > 0
        a, b = f(op, 1000, 1), f(op, 1 << 20, 1)
        assert 0 < a < b
    assert f(2, 1 << 20, 1) > f(1, 1 << 20, 1)  # gradient payload is larger
    assert f(5, 1 << 20, 1) > f(1, 1 << 20, 1)  # the stream adds its extracted arrays
    assert f(1, -1, 1) == 0 and f(1, 1 << 31, 1) == 0
    assert f(3, 100, 0) == 0 and f(9, 100, 1) == 0


def test_status_strings(lib):
    lib.tb_status_str.restype = ctypes.c_char_p
    lib.tb_status_str.argtypes = [ctypes.c_int]
    for s in range(7):
        assert lib.tb_status_str(s).decode().startswith("TB_")


def test_argument_errors_return_before_device_work(lib):
    P, I64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.tb_bbox.argtypes = [P, P, I64, P, P, P, SZ, P, P]
    lib.tb_match.argtypes = [P, I64, P, P, P, SZ, P, P]
    lib.tb_bbox_backward.argtypes = [P, P, P, I64, P, P, SZ, P, P]
    lib.tb_bbox_batched.argtypes = [P, P, P, I64, I64, P, P, P, SZ, P, P]
    for f in (lib.tb_bbox, lib.tb_match, lib.tb_bbox_backward, lib.tb_bbox_batched):
        f.restype = ctypes.c_int
    A = 1 << 20  # fake, aligned addresses: never dereferenced on these paths
    big = 1 << 40
    # sizes
    assert lib.tb_bbox(A, A, -1, A, A, A, big, A, None) == TB_ERR_SIZE
    assert lib.tb_bbox(A, A, 1 << 31, A, A, A, big, A, None) == TB_ERR_SIZE
    assert lib.tb_bbox_batched(A, A, A, 0, 10, A, A, A, big, A, None) == TB_ERR_SIZE
    # nulls
    assert lib.tb_bbox(A, None, 10, A, A, A, big, A, None) == TB_ERR_NULL
    assert lib.tb_bbox(A, A, 10, A, A, None, big, A, None) == TB_ERR_NULL
    assert lib.tb_bbox(A, A, 10, A, A, A, big, None, None) == TB_ERR_NULL
    assert lib.tb_match(None, 10, A, None, A, big, A, None) == TB_ERR_NULL
    assert lib.tb_bbox_backward(A, A, None, 10, A, A, big, A, None) == TB_ERR_NULL
    assert lib.tb_bbox_batched(A, A, None, 3, 10, A, A, A, big, A, None) == TB_ERR_NULL
    # alignment
    assert lib.tb_bbox(A, A + 4, 10, A, A, A, big, A, None) == TB_ERR_ALIGN
    assert lib.tb_bbox(A + 2, A, 10, A, A, A, big, A, None) == TB_ERR_ALIGN
    assert lib.tb_bbox(A, A, 10, A, A, A + 16, big, A, None) == TB_ERR_ALIGN
    assert lib.tb_bbox_batched(A, A, A + 4, 3, 10, A, A, A, big, A, None) == TB_ERR_ALIGN
    # workspace too small
    assert lib.tb_bbox(A, A, 10, A, A, A, 16, A, None) == TB_ERR_WORKSPACE
    assert lib.tb_bbox_backward(A, A, A, 10, A, A, 16, A, None) == TB_ERR_WORKSPACE


def test_compose_argument_errors(lib):
    P, I64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.tb_compose.argtypes = [P, P, I64, P, P, SZ, P, P]
    lib.tb_compose.restype = ctypes.c_int
    A = 1 << 20
    big = 1 << 40
    assert lib.tb_compose(A, A, -1, A, A, big, A, None) == TB_ERR_SIZE
    assert lib.tb_compose(A, None, 10, A, A, big, A, None) == TB_ERR_NULL
    assert lib.tb_compose(A, A, 10, None, A, big, A, None) == TB_ERR_NULL
    assert lib.tb_compose(A, A, 10, A, A, big, None, None) == TB_ERR_NULL
    assert lib.tb_compose(A, A + 4, 10, A, A, big, A, None) == TB_ERR_ALIGN  # rows need 8 bytes
    assert lib.tb_compose(A, A, 10, A, A, 16, A, None) == TB_ERR_WORKSPACE


def test_stream_argument_errors(lib):
    P, I64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    lib.tb_bbox_stream.argtypes = [P, P, I64, P, P, P, SZ, P, P]
    lib.tb_bbox_stream.restype = ctypes.c_int
    A = 1 << 20
    big = 1 << 40
    f = lib.tb_bbox_stream
    assert f(A, A, -1, A, A, A, big, A, None) == TB_ERR_SIZE
    assert f(A, A, 1 << 31, A, A, A, big, A, None) == TB_ERR_SIZE
    assert f(None, A, 10, A, A, A, big, A, None) == TB_ERR_NULL
    assert f(A, None, 10, A, A, A, big, A, None) == TB_ERR_NULL
    assert f(A, A, 10, A, None, A, big, A, None) == TB_ERR_NULL
    assert f(A, A, 10, A, A, A, big, None, None) == TB_ERR_NULL
    assert f(A + 2, A, 10, A, A, A, big, A, None) == TB_ERR_ALIGN
    assert f(A, A + 4, 10, A, A, A, big, A, None) == TB_ERR_ALIGN
    assert f(A, A, 10, A + 2, A, A, big, A, None) == TB_ERR_ALIGN
    assert f(A, A, 10, A, A, A, 16, A, None) == TB_ERR_WORKSPACE
    lib.tb_workspace_bytes.restype = SZ
    lib.tb_workspace_bytes.argtypes = [ctypes.c_int, I64, I64]
    need = lib.tb_workspace_bytes(5, 10, 1)
    assert f(A, A, 10, A, A, A, need - 1, A, None) == TB_ERR_WORKSPACE


def test_variant_table_host_only(tmp_path):
    """The variant table works without a device: defaults, pins, invalid
    variants, save/load round trip, clear."""
    import paper_2205_11659_amd as tb
    tb.tune_clear()
    assert tb.variant_get(tb.OP_BBOX, 1000) == (4, 4, 4)
    assert tb.variant_get(tb.OP_MATCH, 1 << 20) == (8, 8, 4)
    tb.variant_set(tb.OP_BBOX, 1 << 20, (8, 4, 2))
    assert tb.variant_get(tb.OP_BBOX, (1 << 19) + 1) == (8, 4, 2)  # same size class
    assert tb.variant_get(tb.OP_BBOX, (1 << 20) + 1) == (4, 4, 4)
    for bad in ((3, 4, 4), (4, 4, 5), (16, 4, 4)):
        with pytest.raises(tb.TreeBBoxError):
            tb.variant_set(tb.OP_BBOX, 100, bad)
    with pytest.raises(tb.TreeBBoxError):
        tb.variant_set(tb.OP_MATCH, 100, (4, 4, 2))  # matching has no cross pass to vary
    with pytest.raises(tb.TreeBBoxError):
        tb.variant_get(tb.OP_COMPOSE, 100)
    path = tmp_path / "tune.txt"
    tb.tune_save(str(path))
    tb.tune_clear()
    assert tb.variant_get(tb.OP_BBOX, 1 << 20) == (4, 4, 4)
    tb.tune_load(str(path))
    assert tb.variant_get(tb.OP_BBOX, 1 << 20) == (8, 4, 2)
    (tmp_path / "bad.txt").write_text("not a table\n")
    with pytest.raises(tb.TreeBBoxError):
        tb.tune_load(str(tmp_path / "bad.txt"))
    tb.variant_set(tb.OP_BBOX, 1 << 20, None)
    assert tb.variant_get(tb.OP_BBOX, 1 << 20) == (4, 4, 4)
    tb.tune_clear()
    assert len(tb.candidates(tb.OP_BBOX)) == 12 and len(tb.candidates(tb.OP_MATCH)) == 4
