"""GPU parity of tb_reduce_up_f32 (the leaves' fp32 transforms multiplied up
the tree, segment-tree grouping) against the oracle, bit for bit."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import say, to_dev
from test_gpu_compose_f32 import xf_random

pytestmark = pytest.mark.gpu


def check(kind, xf, tag):
    import torch
    import paper_2205_11659_amd as tb
    say(f"[reduce_up_f32] {tag} n={len(kind)}")
    out, st = tb.tb_reduce_up_f32(to_dev(kind), torch.from_numpy(xf).cuda())
    torch.cuda.synchronize()
    want, ost = oracle.reduce_up_f32(kind, xf)
    assert int(st.item()) == ost, (int(st.item()), ost)
    if ost == 0:
        got = out.cpu().numpy()
        bad = np.flatnonzero((got.view(np.uint32) != want.view(np.uint32)).any(1))
        assert len(bad) == 0, f"{tag}: rows differ at {bad[:10]}"


@pytest.mark.parametrize("n", [1, 2, 3, 1023, 1025, 70_001])
def test_random_walks(n):
    kind, _ = gen.walk(n, 64, 0xD320 + n)
    check(kind, xf_random(n, n + 1), "walk cap 64")


@pytest.mark.parametrize("cap", [1, 5000])
def test_deep(cap):
    kind, _ = gen.walk(400_001, cap, 0xD321 + cap)
    check(kind, xf_random(len(kind), cap + 1), f"walk cap {cap}")


def test_chain_around_walk():
    kind, _ = gen.chain_around_walk(100_000, 300_000, 64, 0xD322)
    check(kind, xf_random(len(kind), 11), "chain 100K")


def test_no_leaves_and_malformed():
    kind = np.array([1, 3, 4, 2, 1, 2], np.uint32)
    check(kind, xf_random(len(kind), 12), "no leaves")
    kind, _ = gen.walk(5000, 20, 0xD323)
    check(np.concatenate([kind, [2]]).astype(np.uint32), xf_random(5001, 13), "extra close")
