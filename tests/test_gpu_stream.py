"""GPU parity of tb_bbox_stream (the draw-object stream front end: extract
the tree's elements by stream compaction, run the pipeline on them, write
results back at stream positions) against the oracle, bit for bit, including
the entries at positions outside the tree, which neither side writes."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, same_bits, to_dev

pytestmark = pytest.mark.gpu
T = 1024
CT = 4096  # stream elements per compaction block
SENT_M = -7


def gpu_stream(tag, box, with_match=True):
    import torch
    import paper_2205_11659_amd as tb
    n = tag.shape[0]
    out = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda:0")
    m = torch.full((n,), SENT_M, dtype=torch.int32, device="cuda:0") if with_match else False
    out, m, st = tb.tb_bbox_stream(to_dev(tag), to_dev(box), match=m, out=out)
    torch.cuda.synchronize()
    return (m.cpu().numpy() if with_match else None), out.cpu().numpy(), int(st.item())


def check(tag, box, name, with_match=True):
    say(f"[stream] {name} n={tag.shape[0]} tree={(tag <= 4).sum()}")
    m, out, st = gpu_stream(tag, box, with_match)
    om, oout, ost = oracle.bbox_stream(tag, box)
    assert st == ost, (st, ost)
    if ost:
        return
    if with_match:
        bad = np.nonzero(m != om)[0]
        assert len(bad) == 0, f"{name}: match differs at {bad[:10]}"
    # NaN rows (never written) compare equal bit for bit on both sides
    rows = np.nonzero((out.view(np.uint32) != oout.view(np.uint32)).any(1))[0]
    assert len(rows) == 0, f"{name}: rows differ at {rows[:10]} tags={tag[rows[:10]]}"


def stream(m, n, cap, seed):
    kind, box = gen.walk(m, cap, 7000 + seed)
    tag, sbox, _ = gen.interleave(kind, box, n, 7100 + seed)
    return tag, sbox


@pytest.mark.parametrize("m,n", [(0, 1), (1, 1), (0, 5000), (3, 7), (1000, 1003), (1023, 4096),
                                 (1025, 4097), (4096, 4096), (3000, 3 * CT + 5),
                                 (20_000, 9 * CT - 1)])
def test_sizes(m, n):
    tag, box = stream(m, n, 64, m + n)
    check(tag, box, f"m={m}")


@pytest.mark.parametrize("seed,m,dens,cap", [(1, 200_000, 0.125, 64), (2, 300_000, 0.5, 300),
                                             (3, 100_000, 0.02, 20_000), (4, 250_000, 1.0, 8)])
def test_random_streams(seed, m, dens, cap):
    tag, box = stream(m, int(m / dens), cap, seed)
    check(tag, box, f"dens={dens} cap={cap}")


@pytest.mark.parametrize("depth,walk,dens", [(T, 500, 0.3), (3 * T + 2, 20_000, 0.6),
                                             (70_000, 200_000, 0.25)])
def test_chains(depth, walk, dens):
    # chains deep enough to cross many partitions of the extracted sequence
    kind, box = gen.chain_around_walk(depth, walk, 64, 7200 + depth)
    tag, sbox, _ = gen.interleave(kind, box, int(len(kind) / dens), 7300 + depth)
    check(tag, sbox, f"chain {depth}")


def test_without_match():
    tag, box = stream(50_000, 200_000, 64, 9)
    check(tag, box, "no match", with_match=False)


def test_status_bits():
    tag, box = stream(5000, 20_000, 16, 10)
    bad = tag.copy()
    bad[np.nonzero(tag == gen.OTHER)[0][::97]] = 6
    check(bad, box, "bad tags")
    _, _, st = gpu_stream(bad, box)
    assert st == oracle.BAD_KIND
    t = tag.copy()
    t[np.nonzero(t == 2)[0][0]] = 4  # END_BLEND closing a BEGIN_CLIP (or worse)
    _, _, st = gpu_stream(t, box)
    assert st != 0 and st == oracle.bbox_stream(t, box)[2]
    t = np.array([1, 5, 5, 2, 5, 2] * 1000, np.uint32)
    _, _, st = gpu_stream(t, np.zeros((len(t), 4), np.float32))
    assert st & oracle.UNBALANCED


def test_only_other_elements():
    tag = np.full(3 * CT + 17, gen.OTHER, np.uint32)
    box = np.ones((len(tag), 4), np.float32)
    m, out, st = gpu_stream(tag, box)
    assert st == 0 and (m == SENT_M).all() and np.isnan(out).all()


def test_misaligned_tag_and_kind_arrays():
    """tag / kind arrays need only 4-byte alignment: offset views by one element."""
    import torch
    import paper_2205_11659_amd as tb
    L = tb.lib()
    tag, box = stream(30_000, 70_001, 64, 11)
    n = tag.shape[0]
    say(f"[stream] misaligned n={n}")
    tbuf = to_dev(np.concatenate([np.zeros(1, np.uint32), tag]))
    dbox = to_dev(box)
    out = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda:0")
    m = torch.full((n,), SENT_M, dtype=torch.int32, device="cuda:0")
    st = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    ws, wsb = tb.workspace(tb.OP_BBOX_STREAM, n, 1, tbuf.device)
    rc = L.tb_bbox_stream(tbuf.data_ptr() + 4, dbox.data_ptr(), n, m.data_ptr(), out.data_ptr(),
                          ctypes.c_void_p(ws), wsb, st.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    om, oout, ost = oracle.bbox_stream(tag, box)
    assert int(st.item()) == ost == 0
    assert np.array_equal(m.cpu().numpy(), om) and same_bits(out.cpu().numpy(), oout)
    # the plain forward with a kind array offset by 4 bytes
    kind, kbox = gen.walk(50_001, 64, 12)
    kbuf = to_dev(np.concatenate([np.zeros(1, np.uint32), kind]))
    kdbox = to_dev(kbox)
    n = kind.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda:0")
    m = torch.empty((n,), dtype=torch.int32, device="cuda:0")
    ws, wsb = tb.workspace(tb.OP_BBOX, n, 1, kbuf.device)
    rc = L.tb_bbox(kbuf.data_ptr() + 4, kdbox.data_ptr(), n, m.data_ptr(), out.data_ptr(),
                   ctypes.c_void_p(ws), wsb, st.data_ptr(), None)
    assert rc == 0
    torch.cuda.synchronize()
    om, _, oout, ost = oracle.bbox(kind, kbox)
    assert int(st.item()) == ost == 0
    assert np.array_equal(m.cpu().numpy(), om) and same_bits(out.cpu().numpy(), oout)


def test_repeated_calls_share_workspace():
    """A second, smaller call on the same workspace sees none of the first's
    extracted elements."""
    t1, b1 = stream(60_000, 100_000, 64, 13)
    t2, b2 = stream(2_000, 90_000, 64, 14)
    check(t1, b1, "first")
    check(t2, b2, "second, fewer tree elements")


def test_stream_128m_tree_16m():
    w = gen.stream_config()
    check(w["tag"], w["box"], w["name"])
