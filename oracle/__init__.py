"""ORACLE -- test infrastructure only.

ctypes wrapper over ``tb_oracle.c``, the plain sequential CPU walk.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the
product path never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tb_oracle.c")
LIB_PATH = os.path.join(_HERE, "libtboracle.so")

BAD_KIND, UNBALANCED, KIND_MISMATCH, BAD_OFFSETS = 1, 2, 4, 8

_lib = None


def build():
    """Compile the oracle library in place (gcc -O2, host only)."""
    tmp = LIB_PATH + ".tmp"
    # -ffp-contract=off: every fp32 multiply and add rounds on its own
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp,
                           _SRC, "-lm"])
    os.replace(tmp, LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, U32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32
        L.tbo_bbox.argtypes = [P, P, I64, P, P, P]
        L.tbo_match.argtypes = [P, I64, P, P]
        L.tbo_bbox_f64.argtypes = [P, P, I64, P]
        L.tbo_backward.argtypes = [P, P, P, I64, P]
        L.tbo_sources.argtypes = [P, P, I64, P]
        L.tbo_compose.argtypes = [P, P, I64, P]
        L.tbo_bbox_stream.argtypes = [P, P, I64, P, P]
        L.tbo_match_brackets.argtypes = [P, I64, P, P]
        L.tbo_compose_f32.argtypes = [P, P, I64, P]
        L.tbo_reduce_up_f32.argtypes = [P, P, I64, P]
        for f in (L.tbo_bbox, L.tbo_match, L.tbo_bbox_f64, L.tbo_backward, L.tbo_sources,
                  L.tbo_compose, L.tbo_bbox_stream, L.tbo_match_brackets, L.tbo_compose_f32,
                  L.tbo_reduce_up_f32):
            f.restype = U32
        _lib = L
    return _lib


def _c(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a


def bbox(kind, box):
    """Forward walk. Returns (match int32[n], pm int32[n], out float32[n,4], status)."""
    kind = _c(kind, np.uint32)
    box = _c(box, np.float32).reshape(-1, 4)
    n = kind.shape[0]
    match = np.empty(n, np.int32)
    pm = np.empty(n, np.int32)
    out = np.empty((n, 4), np.float32)
    st = lib().tbo_bbox(kind.ctypes.data, box.ctypes.data, n, match.ctypes.data, pm.ctypes.data,
                        out.ctypes.data)
    return match, pm, out, int(st)


def match(kind):
    kind = _c(kind, np.uint32)
    n = kind.shape[0]
    m = np.empty(n, np.int32)
    pm = np.empty(n, np.int32)
    st = lib().tbo_match(kind.ctypes.data, n, m.ctypes.data, pm.ctypes.data)
    return m, pm, int(st)


def match_brackets(tok):
    """Typed bracket matching: token 0 none, 2t+1 open type t, 2t+2 close
    type t.  Returns (match int32[n], pm int32[n], status)."""
    tok = _c(tok, np.uint32)
    n = tok.shape[0]
    m = np.empty(n, np.int32)
    pm = np.empty(n, np.int32)
    st = lib().tbo_match_brackets(tok.ctypes.data, n, m.ctypes.data, pm.ctypes.data)
    return m, pm, int(st)


def bbox_f64(kind, box):
    kind = _c(kind, np.uint32)
    box = _c(box, np.float64).reshape(-1, 4)
    n = kind.shape[0]
    out = np.empty((n, 4), np.float64)
    st = lib().tbo_bbox_f64(kind.ctypes.data, box.ctypes.data, n, out.ctypes.data)
    return out, int(st)


def backward(kind, box, grad_out):
    kind = _c(kind, np.uint32)
    box = _c(box, np.float32).reshape(-1, 4)
    g = _c(grad_out, np.float32).reshape(-1, 4)
    n = kind.shape[0]
    gi = np.empty((n, 4), np.float32)
    st = lib().tbo_backward(kind.ctypes.data, box.ctypes.data, g.ctypes.data, n, gi.ctypes.data)
    return gi, int(st)


def sources(kind, box):
    kind = _c(kind, np.uint32)
    box = _c(box, np.float32).reshape(-1, 4)
    n = kind.shape[0]
    src = np.empty((n, 4), np.int64)
    st = lib().tbo_sources(kind.ctypes.data, box.ctypes.data, n, src.ctypes.data)
    return src, int(st)


def compose(kind, xf):
    """Transform composition down the tree: xf uint32[n,6] rows [a b c d e f]
    (mod 2^32).  Returns (out uint32[n,6], status)."""
    kind = _c(kind, np.uint32)
    xf = _c(xf, np.uint32).reshape(-1, 6)
    n = kind.shape[0]
    out = np.empty((n, 6), np.uint32)
    st = lib().tbo_compose(kind.ctypes.data, xf.ctypes.data, n, out.ctypes.data)
    return out, int(st)


def compose_f32(kind, xf):
    """fp32 transforms composed down the tree in pointer-jumping order:
    xf float32[n,6] rows [a b c d e f].  Returns (out float32[n,6], status)."""
    kind = _c(kind, np.uint32)
    xf = _c(xf, np.float32).reshape(-1, 6)
    n = kind.shape[0]
    out = np.empty((n, 6), np.float32)
    st = lib().tbo_compose_f32(kind.ctypes.data, xf.ctypes.data, n, out.ctypes.data)
    return out, int(st)


def reduce_up_f32(kind, xf):
    """fp32 transforms of the leaves multiplied up the tree (segment-tree
    grouping).  Returns (out float32[n,6], status)."""
    kind = _c(kind, np.uint32)
    xf = _c(xf, np.float32).reshape(-1, 6)
    n = kind.shape[0]
    out = np.full((n, 6), np.nan, np.float32)
    st = lib().tbo_reduce_up_f32(kind.ctypes.data, xf.ctypes.data, n, out.ctypes.data)
    return out, int(st)


def bbox_stream(tag, box, match_init=None, out_init=None):
    """Stream front end: extract the tree elements (tags 0..4), walk them,
    put each result back at its stream position.  Positions tagged 5 keep
    the values of match_init / out_init (default -7 and NaN, so an untouched
    entry is recognisable).  Returns (match int32[n], out float32[n,4], status)."""
    tag = _c(tag, np.uint32)
    box = _c(box, np.float32).reshape(-1, 4)
    n = tag.shape[0]
    match = np.full(n, -7, np.int32) if match_init is None else np.array(match_init, np.int32)
    out = np.full((n, 4), np.nan, np.float32) if out_init is None else np.array(out_init, np.float32)
    st = lib().tbo_bbox_stream(tag.ctypes.data, box.ctypes.data, n, match.ctypes.data,
                               out.ctypes.data)
    return match, out, int(st)
