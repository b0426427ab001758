"""GPU parity of tb_compose (transforms composed down the tree, a
non-commutative monoid) against the oracle.  The arithmetic is exact modulo
2^32, so every comparison is bit-exact whatever order the parallel steps
group the products in."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu
T = 1024


def gpu_compose(kind, xf):
    import torch
    import paper_2205_11659_amd as tb
    out, st = tb.tb_compose(to_dev(kind), to_dev(xf.view(np.int32)))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32), int(st.item())


def rand_xf(n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 32, size=(n, 6), dtype=np.uint64).astype(np.uint32)


def check(kind, xf, tag):
    say(f"[compose] {tag} n={len(kind)}")
    out, st = gpu_compose(kind, xf)
    oout, ost = oracle.compose(kind, xf)
    assert st == ost, (st, ost)
    if ost == 0:
        bad = np.nonzero((out != oout).any(1))[0]
        assert len(bad) == 0, f"{tag}: rows differ at {bad[:10]} kinds={kind[bad[:10]]}"


@pytest.mark.parametrize("n", [1, 2, 17, 1023, 1024, 1025, 4097, 70_001])
def test_sizes(n):
    kind, _ = gen.walk(n, 64, 6000 + n)
    check(kind, rand_xf(n, n), f"walk n={n}")


@pytest.mark.parametrize("seed,n,cap", [(1, 200_000, 4), (2, 300_000, 300), (3, 150_000, 20_000)])
def test_random_walks(seed, n, cap):
    kind, _ = gen.walk(n, cap, 6100 + seed)
    check(kind, rand_xf(n, 10 + seed), f"walk cap={cap}")


@pytest.mark.parametrize("depth,walk", [(T, 500), (3 * T + 2, 20_000), (70_000, 200_000)])
def test_chains(depth, walk):
    kind, _ = gen.chain_around_walk(depth, walk, 64, 6200 + depth)
    check(kind, rand_xf(len(kind), depth), f"chain {depth}")


def test_chains_scene_16m():
    kind = gen.config(1)["kind"]
    check(kind, rand_xf(len(kind), 99), "16M chains")


def test_empty_and_status():
    out, st = gpu_compose(np.zeros(0, np.uint32), np.zeros((0, 6), np.uint32))
    assert st == 0 and out.shape == (0, 6)
    k, _ = gen.walk(4000, 20, 9)
    for kk in (np.concatenate([k, [7]]), np.concatenate([k, [4]]), np.concatenate([[3], k])):
        kk = kk.astype(np.uint32)
        xf = rand_xf(len(kk), 1)
        _, ost = oracle.compose(kk, xf)
        _, st = gpu_compose(kk, xf)
        assert ost != 0 and st == ost, (ost, st)
