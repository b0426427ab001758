"""GPU parity of tb_match_brackets (typed brackets) against the oracle:
match, pm and status bit for bit, on streams spanning many partitions,
deep chains, mistyped closes, the extreme token values, and every launch
variant."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def gpu_brackets(tok):
    import torch
    import paper_2205_11659_amd as tb
    m, pm, st = tb.tb_match_brackets(to_dev(tok))
    torch.cuda.synchronize()
    return m.cpu().numpy(), pm.cpu().numpy(), int(st.item())


def check(tok, tag, want_status=None):
    """Status always; match and pm whenever the nesting is well formed (a
    mistyped close still matches its open; with UNBALANCED the outputs are
    unspecified)."""
    say(f"[brackets] {tag} n={len(tok)}")
    m, pm, st = gpu_brackets(tok)
    om, opm, ost = oracle.match_brackets(tok)
    if want_status is not None:
        assert ost == want_status, ost
    assert st == ost, (st, ost)
    if ost & 2:
        return
    assert np.array_equal(m, om), f"{tag}: match differs at {np.flatnonzero(m != om)[:10]}"
    assert np.array_equal(pm, opm), f"{tag}: pm differs at {np.flatnonzero(pm != opm)[:10]}"


@pytest.mark.parametrize("n", [1, 2, 5, 1023, 1025, 4099, 70_001])
@pytest.mark.parametrize("ntypes", [1, 4, 1000])
def test_random_streams(n, ntypes):
    check(gen.brackets(n, 64, ntypes, 0xB000 + n + ntypes), f"types={ntypes}", 0)


@pytest.mark.parametrize("cap", [3, 5000, 300_000])
def test_deep(cap):
    check(gen.brackets(700_001, cap, 7, 0xB100 + cap), f"cap={cap}", 0)


def test_chain_of_types():
    depth = 300_000
    t = (np.arange(depth) * 2654435761 % 1_000_003).astype(np.uint32)
    tok = np.concatenate([2 * t + 1, np.zeros(5, np.uint32), (2 * t + 2)[::-1]]).astype(np.uint32)
    check(tok, "typed chain 300K", 0)
    bad = tok.copy()
    bad[len(bad) - 1 - 123_456] += 2  # one close of the wrong type, deep in the chain
    check(bad, "one mistyped close", 4)


def test_mistyped_and_unbalanced():
    check(gen.brackets(200_000, 80, 5, 0xB200, 0.001), "mistyped", 4)
    tok = gen.brackets(50_000, 40, 3, 0xB201)
    check(np.concatenate([[2], tok]).astype(np.uint32), "leading close")
    check(np.concatenate([tok, [7]]).astype(np.uint32), "trailing open")


def test_extreme_tokens():
    big = np.array([0xFFFFFFFD, 0, 0xFFFFFFFE, 0xFFFFFFFF, 2], np.uint32)
    check(big, "largest types")  # 0xFFFFFFFF opens a type no token closes
    tok = np.tile(np.array([0xFFFFFFFD, 1, 2, 0xFFFFFFFE], np.uint32), 5000)
    check(tok, "largest valid type", 0)


def test_every_variant():
    import paper_2205_11659_amd as tb
    tok = gen.brackets(300_003, 3000, 9, 0xB300, 0.0005)
    try:
        for v in tb.candidates(tb.OP_MATCH):
            tb.variant_set(tb.OP_MATCH, len(tok), v)
            check(tok, f"variant {v}", 4)
    finally:
        tb.tune_clear()
