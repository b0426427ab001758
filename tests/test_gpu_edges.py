"""GPU parity on edge cases: partition-aligned and misaligned chains,
degenerate and infinite box coordinates, scene boundaries that fall on
partition and thread boundaries, a null match pointer, and the Fig. 1 `pm`
output on a large scene.  Every comparison is bit-exact against the oracle."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import gpu_batched, gpu_bbox, gpu_match, same_bits, say, to_dev

pytestmark = pytest.mark.gpu

T = 1024  # partition size of the kernels (only used to place boundaries)


def chain(depth, rng, leaves_mid=0):
    """`depth` alternating clip/blend opens, `leaves_mid` leaves, matching closes."""
    opens = np.where(np.arange(depth) % 2 == 0, 1, 3).astype(np.uint32)
    closes = np.where(opens[::-1] == 1, 2, 4).astype(np.uint32)
    kind = np.concatenate([opens, np.zeros(leaves_mid, np.uint32), closes])
    box = rng.uniform(0, 100, size=(len(kind), 2)).astype(np.float32)
    wh = rng.uniform(1, 400, size=(len(kind), 2)).astype(np.float32)
    return kind, np.concatenate([box, box + wh], axis=1).astype(np.float32)


def check(kind, box, tag):
    say(f"[edge] {tag} n={len(kind)}")
    m, out, st = gpu_bbox(kind, box)
    om, _, oout, ost = oracle.bbox(kind, box)
    assert st == ost, (st, ost)
    if ost == 0:
        assert np.array_equal(m, om), f"{tag}: match"
        assert same_bits(out, oout), f"{tag}: boxes"


@pytest.mark.parametrize("depth", [T // 2 - 1, T // 2, T // 2 + 1, T, T + 1, 3 * T + 2])
@pytest.mark.parametrize("lead", [0, 1, 3])
def test_chain_alignment(depth, lead):
    """Chains whose opens end on, just before and just after partition and
    thread boundaries (`lead` leaves shift the whole chain)."""
    rng = np.random.default_rng(depth * 7 + lead)
    k, b = chain(depth, rng, leaves_mid=lead)
    pre_k = np.zeros(lead, np.uint32)
    pre_b = rng.uniform(0, 500, size=(lead, 4)).astype(np.float32)
    pre_b[:, 2:] = pre_b[:, :2] + 50
    check(np.concatenate([pre_k, k]), np.concatenate([pre_b, b]), f"chain {depth} lead {lead}")


def test_degenerate_and_infinite_boxes():
    """Coordinates from a small set with infinities, equal, touching, zero-width
    and inverted boxes (inverted inputs are simply empty)."""
    rng = np.random.default_rng(5)
    vals = np.array([-np.inf, -7.0, 0.0, 1.0, 2.0, 3.5, np.inf], np.float32)
    for cap in (4, 64, 1000):
        kind, _ = gen.walk(60_000, cap, 300 + cap)
        box = vals[rng.integers(0, len(vals), size=(len(kind), 4))]
        check(kind, box, f"degenerate cap={cap}")


def test_null_match_pointer():
    import torch
    import paper_2205_11659_amd as tb
    kind, box = gen.walk(100_000, 64, 77, gen.BOX_NESTED_ALL)
    out, m, st = tb.tb_bbox(to_dev(kind), to_dev(box), match=False)
    torch.cuda.synchronize()
    assert m is None and int(st.item()) == 0
    _, _, oout, _ = oracle.bbox(kind, box)
    assert same_bits(out.cpu().numpy(), oout)


def test_pm_on_chains_scene():
    """Fig. 1's top-of-stack output over chains 100,000 deep."""
    kind = gen.config(1)["kind"]
    say(f"[edge] pm n={len(kind)}")
    m, pm, st = gpu_match(kind)
    om, opm, ost = oracle.match(kind)
    assert st == 0 and ost == 0
    assert np.array_equal(m, om) and np.array_equal(pm, opm)


def scenes_to_batch(parts):
    kind = np.concatenate([p[0] for p in parts]).astype(np.uint32)
    box = np.concatenate([p[1] for p in parts]).astype(np.float32)
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]).astype(np.int64)
    return kind, box, off


def check_batched(kind, box, off, tag, bad=()):
    say(f"[edge] batched {tag} n={len(kind)} scenes={len(off) - 1}")
    m, out, st = gpu_batched(kind, box, off)
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        om, _, oout, ost = oracle.bbox(kind[a:b], box[a:b])
        assert st[s] == ost, (tag, s, st[s], ost)
        if s in bad:
            assert ost != 0
            continue
        assert np.array_equal(m[a:b], om), f"{tag}: scene {s} match"
        assert same_bits(out[a:b], oout), f"{tag}: scene {s} boxes"


def test_batched_boundaries_on_partitions_and_threads():
    """Scene starts at exact partition starts, at every position inside a
    thread, and scenes of one and two elements."""
    rng = np.random.default_rng(11)
    parts = []
    sizes = [T, T, 1, 2, T - 1, 3, 2 * T + 2, 5, 6, 7, 4 * T, 1, 1, 2]
    for i, n in enumerate(sizes):
        if n == 1:
            k = np.zeros(1, np.uint32)
            b = rng.uniform(0, 10, size=(1, 4)).astype(np.float32)
        elif n == 2:
            k = np.array([1, 2], np.uint32)
            b = rng.uniform(0, 10, size=(2, 4)).astype(np.float32)
        else:
            k, b = gen.walk(n, 16, 500 + i, gen.BOX_NESTED_ALL)
        parts.append((k, b))
    kind, box, off = scenes_to_batch(parts)
    check_batched(kind, box, off, "aligned/misaligned")


def test_batched_deep_scene_between_shallow_ones():
    rng = np.random.default_rng(12)
    parts = [gen.walk(5000, 8, 600, gen.BOX_NESTED_ALL), chain(60_000, rng, leaves_mid=3),
             gen.walk(7001, 300, 601, gen.BOX_NESTED_ALL), chain(T, rng), gen.walk(3, 2, 602)]
    kind, box, off = scenes_to_batch(parts)
    check_batched(kind, box, off, "deep middle scene")


def test_batched_unbalanced_scene_on_partition_boundary():
    """A scene ending in an extra close exactly at a partition boundary, and
    one starting with an unclosed open; the other scenes stay exact."""
    rng = np.random.default_rng(13)
    k0, b0 = gen.walk(T - 1, 16, 700, gen.BOX_NESTED_ALL)
    k0 = np.concatenate([k0, [2]]).astype(np.uint32)  # extra close at element T-1
    b0 = np.concatenate([b0, np.zeros((1, 4), np.float32)])
    k2, b2 = gen.walk(3000, 16, 702, gen.BOX_NESTED_ALL)
    k2 = np.concatenate([[3], k2]).astype(np.uint32)  # never-closed blend open
    b2 = np.concatenate([np.zeros((1, 4), np.float32), b2])
    parts = [(k0, b0), gen.walk(2 * T, 16, 701, gen.BOX_NESTED_ALL), (k2, b2),
             chain(500, rng)]
    kind, box, off = scenes_to_batch(parts)
    check_batched(kind, box, off, "unbalanced scenes", bad=(0, 2))


@pytest.mark.parametrize("depth", [T // 2, T, 3 * T + 2])
def test_match_only_chains(depth):
    """The matching-only path (its own thread layout) on chains crossing
    partition boundaries."""
    rng = np.random.default_rng(depth)
    k, _ = chain(depth, rng, leaves_mid=5)
    k = np.concatenate([gen.walk(777, 9, 31)[0], k, gen.walk(1001, 40, 32)[0]]).astype(np.uint32)
    say(f"[edge] match chain {depth} n={len(k)}")
    m, pm, st = gpu_match(k)
    om, opm, ost = oracle.match(k)
    assert st == 0 and ost == 0
    assert np.array_equal(m, om) and np.array_equal(pm, opm)


def test_match_only_status_bits():
    k, _ = gen.walk(5000, 30, 1)
    closes = np.nonzero(k == 2)[0]
    k1 = k.copy(); k1[2500] = 9
    k2 = np.concatenate([k, [2]]).astype(np.uint32)
    k3 = np.concatenate([[1], k]).astype(np.uint32)
    k4 = k.copy(); k4[closes[len(closes) // 2]] = 4
    for kk in (k1, k2, k3, k4):
        _, _, ost = oracle.match(kk)
        _, _, st = gpu_match(kk)
        assert ost != 0 and st == ost, (ost, st)
