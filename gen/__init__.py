"""Seeded synthetic scene inputs (shared by the oracle tests, the GPU tests and
the benchmark).  Thin ctypes wrapper over ``treegen.c``; no bounding-box
arithmetic lives here.

Element kinds: 0 LEAF, 1 BEGIN_CLIP, 2 END_CLIP, 3 BEGIN_BLEND, 4 END_BLEND.
Boxes are float32 rows (x0, y0, x1, y1); rows other than LEAF / BEGIN_CLIP are 0.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "treegen.c")
LIB_PATH = os.path.join(_HERE, "libtreegen.so")

BOX_INDEP, BOX_NESTED, BOX_GRID, BOX_NESTED_ALL, BOX_INSET, BOX_INSET_ND = 0, 1, 2, 3, 4, 5
SEED_BASE = 0x7B0B0000

_lib = None


def build():
    """Compile the generator library in place (gcc, host only)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-shared", "-fPIC",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, U64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
        L.tbg_walk.argtypes = [P, P, I64, I64, U64, I32]
        L.tbg_walk_with_chains.argtypes = [P, P, I64, I64, I64, I64, I64, U64, I32]
        L.tbg_chain_around_walk.argtypes = [P, P, I64, I64, I64, U64, I32]
        L.tbg_batch.argtypes = [P, P, P, I64, ctypes.c_double, ctypes.c_double, I64, I64, U64, I32]
        L.tbg_batch.restype = I64
        L.tbg_normal.argtypes = [P, I64, U64]
        L.tbg_raw.argtypes = [P, I64, U64]
        L.tbg_interleave.argtypes = [P, P, I64, I64, ctypes.c_uint32, U64, P, P]
        L.tbg_interleave.restype = ctypes.c_int
        L.tbg_brackets.argtypes = [P, I64, I64, ctypes.c_uint32, ctypes.c_double, U64]
        L.tbg_brackets.restype = ctypes.c_int
        L.tbg_splitmix64.argtypes = [U64]
        L.tbg_splitmix64.restype = U64
        for f in (L.tbg_walk, L.tbg_walk_with_chains, L.tbg_chain_around_walk):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _alloc(n):
    return np.zeros(n, dtype=np.uint32), np.zeros((n, 4), dtype=np.float32)


def walk(n, cap, seed, box_mode=BOX_INDEP):
    """Balanced random walk of n elements with depth cap `cap`."""
    kind, box = _alloc(n)
    rc = lib().tbg_walk(kind.ctypes.data, box.ctypes.data, n, cap, seed, box_mode)
    assert rc == 0, rc
    return kind, box


def walk_with_chains(n_walk, cap, n_chains, depth, leaves, seed, box_mode=BOX_INDEP):
    n = n_walk + n_chains * (2 * depth + leaves)
    kind, box = _alloc(n)
    rc = lib().tbg_walk_with_chains(kind.ctypes.data, box.ctypes.data, n_walk, cap, n_chains,
                                    depth, leaves, seed, box_mode)
    assert rc == 0, rc
    return kind, box


def chain_around_walk(depth, n_walk, cap, seed, box_mode=BOX_NESTED):
    n = 2 * depth + n_walk
    kind, box = _alloc(n)
    rc = lib().tbg_chain_around_walk(kind.ctypes.data, box.ctypes.data, depth, n_walk, cap, seed,
                                     box_mode)
    assert rc == 0, rc
    return kind, box


def batch(num_scenes, lg_lo, lg_hi, cap_lo, cap_hi, seed, box_mode=BOX_INDEP):
    offsets = np.zeros(num_scenes + 1, dtype=np.int64)
    total = lib().tbg_batch(None, None, offsets.ctypes.data, num_scenes, lg_lo, lg_hi, cap_lo,
                            cap_hi, seed, box_mode)
    kind, box = _alloc(int(total))
    t2 = lib().tbg_batch(kind.ctypes.data, box.ctypes.data, offsets.ctypes.data, num_scenes,
                         lg_lo, lg_hi, cap_lo, cap_hi, seed, box_mode)
    assert t2 == total
    return kind, box, offsets


OTHER = 5  # tag of a stream element outside the tree


def interleave(kind, box, n, seed, other=OTHER):
    """Place the tree (kind, box) of m elements, in order, on a uniformly
    random m-subset of n stream positions; the rest get tag `other` and a
    random finite box.  Returns (tag, box, positions)."""
    kind = np.ascontiguousarray(kind, dtype=np.uint32)
    box = np.ascontiguousarray(box, dtype=np.float32).reshape(-1, 4)
    m = kind.shape[0]
    tag, sbox = _alloc(n)
    rc = lib().tbg_interleave(kind.ctypes.data, box.ctypes.data, m, n, other, seed,
                              tag.ctypes.data, sbox.ctypes.data)
    assert rc == 0, rc
    pos = np.flatnonzero(tag != other) if other > 4 else None
    return tag, sbox, pos


def brackets(n, cap, ntypes, seed, p_bad=0.0):
    """Typed bracket tokens (0 none, 2t+1 open type t, 2t+2 close type t)
    from a depth-capped random walk; p_bad mistypes that fraction of closes."""
    tok = np.zeros(n, dtype=np.uint32)
    rc = lib().tbg_brackets(tok.ctypes.data, n, cap, ntypes, p_bad, seed)
    assert rc == 0, rc
    return tok


def normal(n, seed):
    out = np.zeros(n, dtype=np.float32)
    lib().tbg_normal(out.ctypes.data, n, seed)
    return out


def raw(n, seed):
    out = np.zeros(n, dtype=np.uint64)
    lib().tbg_raw(out.ctypes.data, n, seed)
    return out


def splitmix64(x):
    return int(lib().tbg_splitmix64(x))


# ---------------------------------------------------------------- workloads
# The five synthetic workloads.  Each returns a dict with at least kind, box.
C1_CHAINS, C1_DEPTH, C1_LEAVES = 16, 100_000, 8


def config(i, nested_boxes=False):
    """Workload i.  nested_boxes=True swaps the independent boxes of the
    walks for BOX_INSET boxes (non-empty clip contexts, 5% of walk clips
    disjoint from their parent); the 2^27 chain scene always uses them."""
    seed = SEED_BASE + i
    if i == 0:  # 65,536 elements, depth cap 64
        k, b = walk(65536, 64, seed, BOX_INSET if nested_boxes else BOX_INDEP)
        return dict(name="scene-64K-cap64", kind=k, box=b)
    if i == 1:  # 2^24: depth<=16 walk with 16 embedded chains of depth 100,000
        n = 1 << 24
        n_walk = n - C1_CHAINS * (2 * C1_DEPTH + C1_LEAVES)
        k, b = walk_with_chains(n_walk, 16, C1_CHAINS, C1_DEPTH, C1_LEAVES, seed,
                                BOX_INSET if nested_boxes else BOX_INDEP)
        return dict(name="scene-16M-chains100K", kind=k, box=b)
    if i == 2:  # 2^27: chain of depth 2^25 around a 2^26 cap-64 walk
        k, b = chain_around_walk(1 << 25, 1 << 26, 64, seed, BOX_INSET)
        return dict(name="scene-128M-chain32M", kind=k, box=b)
    if i == 3:  # 2048 ragged scenes, sizes 2^U[6,18], caps U{4..4096}
        k, b, off = batch(2048, 6.0, 18.0, 4, 4096, seed,
                          BOX_INSET if nested_boxes else BOX_INDEP)
        return dict(name="batch-2048-ragged", kind=k, box=b, offsets=off)
    if i == 4:  # 2^24, cap 256, grid coordinates, N(0,1) upstream gradient
        n = 1 << 24
        k, b = walk(n, 256, seed, BOX_GRID)
        g = normal(4 * n, splitmix64(seed)).reshape(n, 4)
        return dict(name="scene-16M-cap256-grad", kind=k, box=b, grad=g)
    raise ValueError(i)


def stream_config(n=1 << 27, m=1 << 24, cap=64, seed=SEED_BASE + 16):
    """Draw-object stream: a cap-`cap` random walk of m tree elements spread
    over n stream positions (density m/n), every other position tagged OTHER."""
    k, b = walk(m, cap, seed, BOX_INDEP)
    tag, sbox, _ = interleave(k, b, n, splitmix64(seed))
    return dict(name=f"stream-{n >> 20}M-tree{m >> 20}M" if m >= 1 << 20 else f"stream-{n}-tree{m}",
                tag=tag, box=sbox, m=m)
