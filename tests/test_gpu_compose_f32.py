"""GPU parity of tb_compose_f32 (fp32 transforms composed down the tree in
pointer-jumping order) against the oracle, bit for bit: products round, so
this checks the combine order as well as the arithmetic."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def xf_random(n, seed):
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0, 2 * np.pi, n)
    s = rng.uniform(0.5, 2.0, n)
    return np.stack([s * np.cos(ang), -s * np.sin(ang), rng.uniform(-100, 100, n),
                     s * np.sin(ang), s * np.cos(ang), rng.uniform(-100, 100, n)], 1).astype(np.float32)


def check(kind, xf, tag):
    import torch
    import paper_2205_11659_amd as tb
    say(f"[compose_f32] {tag} n={len(kind)}")
    out, st = tb.tb_compose_f32(to_dev(kind), torch.from_numpy(xf).cuda())
    torch.cuda.synchronize()
    want, ost = oracle.compose_f32(kind, xf)
    assert int(st.item()) == ost, (int(st.item()), ost)
    if ost == 0:
        got = out.cpu().numpy()
        bad = np.flatnonzero((got.view(np.uint32) != want.view(np.uint32)).any(1))
        assert len(bad) == 0, f"{tag}: rows differ at {bad[:10]}"


@pytest.mark.parametrize("n", [1, 2, 1023, 1025, 70_001])
def test_random_walks(n):
    kind, _ = gen.walk(n, 64, 0xF320 + n)
    check(kind, xf_random(n, n), "walk cap 64")


@pytest.mark.parametrize("cap", [1, 5000])
def test_deep(cap):
    kind, _ = gen.walk(300_000, cap, 0xF321 + cap)
    check(kind, xf_random(len(kind), cap), f"walk cap {cap}")


def test_chain_around_walk():
    kind, _ = gen.chain_around_walk(100_000, 200_000, 64, 0xF322)
    check(kind, xf_random(len(kind), 7), "chain 100K")


def test_empty_and_malformed():
    import torch
    import paper_2205_11659_amd as tb
    out, st = tb.tb_compose_f32(to_dev(np.zeros(0, np.uint32)), torch.zeros((0, 6), device="cuda"))
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and out.shape == (0, 6)
    kind, _ = gen.walk(5000, 20, 0xF323)
    check(np.concatenate([[1], kind]).astype(np.uint32), xf_random(5001, 8), "unclosed open")
    check(np.concatenate([kind, [9]]).astype(np.uint32), xf_random(5001, 9), "bad kind")
