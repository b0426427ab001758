"""GPU parity of tb_bbox_backward (and TreeBBoxFn) against the oracle's
reference gradient: bit-exact, since both sum the same 64-bit fixed-point
contributions and round once to fp32.  The oracle gradient itself is pinned
to fp64 central differences in test_oracle_grad.py."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import gpu_bbox, same_bits, say, to_dev

pytestmark = pytest.mark.gpu


def nested_grid(n, cap, seed, step=8.0):
    """Boxes nested in their clip ancestor on a grid: non-empty clips and
    frequent ties, so many coordinates route to ancestors and across rows."""
    kind, _ = gen.walk(n, cap, seed, gen.BOX_GRID)
    rng = np.random.default_rng(seed)
    box = np.zeros((n, 4), np.float32)
    stack = []
    for i, k in enumerate(kind):
        if k in (0, 1):
            a = box[stack[-1]] if stack else np.array([0, 0, 64 * step, 64 * step], np.float32)
            x0 = a[0] + step * rng.integers(-1, 3)
            y0 = a[1] + step * rng.integers(-1, 3)
            box[i] = [x0, y0, x0 + step * rng.integers(1, 8), y0 + step * rng.integers(1, 8)]
        if k == 1:
            stack.append(i)
        elif k == 2:
            stack.pop()
    return kind, box


def gpu_backward(kind, box, g):
    import torch
    import paper_2205_11659_amd as tb
    gi, st = tb.tb_bbox_backward(to_dev(kind), to_dev(box), to_dev(g))
    torch.cuda.synchronize()
    return gi.cpu().numpy(), int(st.item())


def check(kind, box, g, tag):
    say(f"[bwd] {tag} n={len(kind)}")
    gi, st = gpu_backward(kind, box, g)
    ogi, ost = oracle.backward(kind, box, g)
    assert st == 0 and ost == 0
    bad = np.nonzero((gi.view(np.uint32) != ogi.view(np.uint32)).any(1))[0]
    assert len(bad) == 0, f"{tag}: grad differs at rows {bad[:10]} gpu={gi[bad[:3]]} cpu={ogi[bad[:3]]}"
    return gi


@pytest.mark.parametrize("n,cap,seed", [(1, 4, 1), (7, 4, 2), (1023, 12, 3), (1025, 12, 4),
                                        (5000, 12, 5), (40_000, 40, 6), (150_000, 300, 7)])
def test_backward_nested(n, cap, seed):
    kind, box = nested_grid(n, cap, 5100 + seed)
    g = gen.normal(4 * n, 5200 + seed).reshape(n, 4)
    gi = check(kind, box, g, f"nested cap={cap}")
    assert (gi != 0).any() or n < 10


def test_backward_chain():
    kind, box = gen.chain_around_walk(6000, 20_000, 30, 5300, gen.BOX_INSET_ND)
    n = len(kind)
    g = gen.normal(4 * n, 5301).reshape(n, 4)
    gi = check(kind, box, g, "chain 6000")
    assert (gi != 0).sum() > n // 4  # the inset boxes route from most rows


def test_backward_workload_16m():
    c = gen.config(4)
    check(c["kind"], c["box"], c["grad"], "16M cap256 grid")


def test_backward_all_leaves():
    n = 3000
    kind = np.zeros(n, np.uint32)
    _, box = gen.walk(n, 0, 5400, gen.BOX_GRID)
    g = gen.normal(4 * n, 5401).reshape(n, 4)
    check(kind, box, g, "all leaves")


def test_autograd_function():
    import torch
    import paper_2205_11659_amd as tb
    kind, box = nested_grid(20_000, 30, 5500)
    n = len(kind)
    g = gen.normal(4 * n, 5501).reshape(n, 4)
    bt = to_dev(box).requires_grad_(True)
    out = tb.bbox(to_dev(kind), bt)
    out.backward(to_dev(g))
    torch.cuda.synchronize()
    _, _, oout, _ = oracle.bbox(kind, box)
    ogi, _ = oracle.backward(kind, box, g)
    assert same_bits(out.detach().cpu().numpy(), oout)
    assert same_bits(bt.grad.cpu().numpy(), ogi)


def test_signed_zero_ties():
    """-0 and +0 compare equal: where they meet, the route goes to the lower
    index as at any tie (the payload orders -0 as +0), and an output row's
    zero may carry either sign, so rows are compared by value here."""
    kind, box = nested_grid(20_000, 30, 5500, step=8.0)
    box = box - np.float32(64.0)  # many coordinates exactly 0 on the grid
    rng = np.random.default_rng(5501)
    zero = box == 0
    assert zero.sum() > 1000
    box[zero & (rng.random(box.shape) < 0.5)] = np.float32(-0.0)
    assert np.signbit(box[box == 0]).any() and (~np.signbit(box[box == 0])).any()
    n = len(kind)
    g = gen.normal(4 * n, 5502).reshape(n, 4)
    check(kind, box, g, "signed zeros")
    m, out, st = gpu_bbox(kind, box)
    om, _, oout, ost = oracle.bbox(kind, box)
    assert st == 0 and ost == 0
    assert np.array_equal(m, om)
    assert np.array_equal(out, oout)  # -0 == +0
