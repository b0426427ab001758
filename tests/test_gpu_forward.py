"""GPU parity of tb_bbox / tb_match / tb_bbox_batched against the CPU oracle.

Matching is integer work and fp32 max/min never rounds, so every comparison
is bit-exact.  Sizes span one and many 1024-element partitions with ragged
tails; the chain cases pop stack levels pushed thousands of partitions
earlier."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import gpu_batched, gpu_bbox, gpu_match, same_bits, say

pytestmark = pytest.mark.gpu


def check_bbox(kind, box, tag):
    say(f"[bbox] {tag} n={len(kind)}")
    m, out, st = gpu_bbox(kind, box)
    om, _, oout, ost = oracle.bbox(kind, box)
    assert ost == 0 and st == 0, (ost, st)
    bad = np.nonzero(m != om)[0]
    assert len(bad) == 0, f"{tag}: match differs at {bad[:10]} gpu={m[bad[:10]]} cpu={om[bad[:10]]}"
    badb = np.nonzero((out.view(np.uint32) != oout.view(np.uint32)).any(1))[0]
    assert len(badb) == 0, f"{tag}: box differs at {badb[:10]} kinds={kind[badb[:10]]}"


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 1023, 1024, 1025, 2047, 2048, 4097, 9999])
def test_small_sizes(n):
    kind, box = gen.walk(n, 64, 7000 + n, gen.BOX_NESTED_ALL)
    check_bbox(kind, box, f"walk n={n}")


def test_empty():
    m, out, st = gpu_bbox(np.zeros(0, np.uint32), np.zeros((0, 4), np.float32))
    assert st == 0 and m.shape == (0,) and out.shape == (0, 4)


@pytest.mark.parametrize("seed,n,cap", [(1, 50_000, 1), (2, 120_000, 8), (3, 200_000, 64),
                                        (4, 300_001, 1000), (5, 150_000, 5000),
                                        (6, 100_000, 100_000)])
def test_random_walks(seed, n, cap):
    kind, box = gen.walk(n, cap, 8000 + seed, gen.BOX_NESTED_ALL)
    check_bbox(kind, box, f"walk cap={cap}")


@pytest.mark.parametrize("depth,walk", [(3000, 20000), (20000, 5000), (70_000, 200_000)])
def test_chain_around_walk(depth, walk):
    kind, box = gen.chain_around_walk(depth, walk, 64, 9000 + depth, gen.BOX_NESTED_ALL)
    check_bbox(kind, box, f"chain depth={depth}")


def test_walk_with_chains():
    kind, box = gen.walk_with_chains(300_000, 16, 5, 20_000, 8, 91, gen.BOX_NESTED_ALL)
    check_bbox(kind, box, "walk+5 chains")


def test_workload_64k():
    for nested in (False, True):
        c = gen.config(0, nested_boxes=nested)
        check_bbox(c["kind"], c["box"], f"64K nested={nested}")


def test_workload_16m_chains():
    c = gen.config(1)
    check_bbox(c["kind"], c["box"], "16M chains")


def test_workload_128m_deep_chain():
    c = gen.config(2)
    check_bbox(c["kind"], c["box"], "128M chain 2^25")


@pytest.mark.parametrize("seed,n,cap", [(1, 1000, 3), (2, 70_000, 64), (3, 200_000, 20_000)])
def test_match_only(seed, n, cap):
    kind, _ = gen.walk(n, cap, 9500 + seed)
    say(f"[match] n={n}")
    m, pm, st = gpu_match(kind)
    om, opm, ost = oracle.match(kind)
    assert st == 0 and ost == 0
    assert np.array_equal(m, om) and np.array_equal(pm, opm)


def check_batched(kind, box, off, tag):
    say(f"[batched] {tag} n={len(kind)} scenes={len(off) - 1}")
    m, out, st = gpu_batched(kind, box, off)
    assert (st == 0).all(), np.nonzero(st)
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        om, _, oout, ost = oracle.bbox(kind[a:b], box[a:b])
        assert ost == 0
        assert np.array_equal(m[a:b], om), f"{tag}: scene {s} match"
        assert same_bits(out[a:b], oout), f"{tag}: scene {s} boxes"


@pytest.mark.parametrize("seed", range(3))
def test_batched_small(seed):
    kind, box, off = gen.batch(40 + 30 * seed, 0.0, 12.0, 1, 300, 9700 + seed, gen.BOX_NESTED_ALL)
    check_batched(kind, box, off, f"seed {seed}")


def test_batched_empty_scenes():
    kind, box, off = gen.batch(20, 3.0, 9.0, 2, 40, 9800, gen.BOX_NESTED_ALL)
    off2 = np.concatenate([[0, 0], off[1:5], [off[4]], off[5:]]).astype(np.int64)
    check_batched(kind, box, off2, "with empty scenes")


@pytest.mark.parametrize("n", [1000, 5000, 300_001])
def test_single_scene_instances_agree(n):
    """tb_bbox runs kernel instances compiled without scene offsets; a batched
    call with one scene runs the instances that search them.  Both must give
    the same bits, and the same status for a malformed scene (whose other
    outputs are unspecified)."""
    kind, box = gen.walk(n, 64, 9900 + n, gen.BOX_NESTED_ALL)
    bad = kind.copy()
    bad[n // 3] = 2  # an extra END_CLIP
    for tag, k in (("well formed", kind), ("malformed", bad)):
        say(f"[single vs batched] {tag} n={n}")
        m1, o1, s1 = gpu_bbox(k, box)
        m2, o2, s2 = gpu_batched(k, box, np.array([0, n], np.int64))
        assert s1 == int(s2[0]), (tag, s1, s2)
        if tag == "well formed":
            assert s1 == 0
            assert np.array_equal(m1, m2) and same_bits(o1, o2), tag
        else:
            assert s1 != 0


def test_batched_workload_2048():
    c = gen.config(3)
    check_batched(c["kind"], c["box"], c["offsets"], "2048 ragged")


def test_batched_bad_scene_is_isolated():
    kind, box, off = gen.batch(30, 6.0, 10.0, 2, 50, 9900, gen.BOX_NESTED_ALL)
    kind = kind.copy()
    bad = 7
    a = off[bad]
    kind[a] = 1  # an extra open at the start of scene 7
    m, out, st = gpu_batched(kind, box, off)
    assert st[bad] & 2, st
    for s in range(len(off) - 1):
        if s == bad:
            continue
        assert st[s] == 0, (s, st[s])
        x, y = off[s], off[s + 1]
        om, _, oout, _ = oracle.bbox(kind[x:y], box[x:y])
        assert np.array_equal(m[x:y], om) and same_bits(out[x:y], oout), s


def test_malformed_status_bits():
    cases = []
    k, b = gen.walk(5000, 30, 1)
    k1 = k.copy(); k1[2500] = 9                       # bad kind
    k2 = k.copy(); k2 = np.concatenate([k2, [2]]).astype(np.uint32)   # trailing extra close
    k3 = np.concatenate([[1], k]).astype(np.uint32)    # leading unclosed open
    closes = np.nonzero(k == 2)[0]
    k4 = k.copy(); k4[closes[len(closes) // 2]] = 4    # END_BLEND closing a BEGIN_CLIP
    for kk in (k1, k2, k3, k4):
        bb = np.zeros((len(kk), 4), np.float32)
        _, _, _, ost = oracle.bbox(kk, bb)
        _, _, st = gpu_bbox(kk, bb)
        assert ost != 0 and st == ost, (ost, st)


def test_deterministic():
    kind, box = gen.walk(400_000, 300, 42, gen.BOX_NESTED_ALL)
    r1 = gpu_bbox(kind, box)
    r2 = gpu_bbox(kind, box)
    assert np.array_equal(r1[0], r2[0]) and same_bits(r1[1], r2[1])
