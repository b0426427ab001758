"""The seeded input generator: determinism, its published RNG definitions,
and the shape statistics of each workload (no GPU)."""
import numpy as np

import brute
import gen

M64 = (1 << 64) - 1


def _splitmix(state):
    state = (state + 0x9E3779B97F4A7C15) & M64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return state, z ^ (z >> 31)


def _xoshiro_stream(seed, n):
    st, s = seed, []
    for _ in range(4):
        st, v = _splitmix(st)
        s.append(v)
    rotl = lambda x, k: ((x << k) | (x >> (64 - k))) & M64
    out = []
    for _ in range(n):
        out.append(rotl((s[1] * 5) & M64, 7) * 9 & M64)
        t = (s[1] << 17) & M64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = rotl(s[3], 45)
    return out


def test_rng_matches_published_definitions():
    for seed in (0, 1, gen.SEED_BASE, 0xDEADBEEFCAFEF00D):
        assert [int(v) for v in gen.raw(16, seed)] == _xoshiro_stream(seed, 16)
        assert gen.splitmix64(seed) == _splitmix(seed)[1]


def test_deterministic():
    a = gen.walk(10000, 64, 5)
    b = gen.walk(10000, 64, 5)
    c = gen.walk(10000, 64, 6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])


def test_walk_shape():
    kind, box = gen.walk(65536, 64, gen.SEED_BASE)
    d = brute.depth_before(kind)
    assert d.max() <= 64 and d.min() >= 0
    final = d[-1] + (1 if kind[-1] in (1, 3) else (-1 if kind[-1] in (2, 4) else 0))
    assert final == 0
    frac = np.bincount(kind, minlength=5) / len(kind)
    assert 0.45 < frac[0] < 0.56 and 0.2 < frac[1] + frac[3] < 0.3
    assert (box[~np.isin(kind, [0, 1])] == 0).all()
    assert (box[np.isin(kind, [0, 1]), 2] >= box[np.isin(kind, [0, 1]), 0]).all()


def test_chain_builders_small():
    k, b = gen.walk_with_chains(5000, 16, 3, 500, 8, 1)
    assert len(k) == 5000 + 3 * 1008
    d = brute.depth_before(k)
    assert d.max() >= 500 and d.min() >= 0
    k, b = gen.chain_around_walk(300, 2000, 64, 2)
    assert len(k) == 2600 and (k[:300] == np.where(np.arange(300) % 2, 3, 1)).all()
    assert np.isin(k[-300:], [2, 4]).all()


def test_batch_offsets():
    k, b, off = gen.batch(50, 6.0, 10.0, 4, 64, 3)
    assert off[0] == 0 and off[-1] == len(k) and (np.diff(off) >= 64).all()
    for s in range(50):
        seg = k[off[s]:off[s + 1]]
        d = brute.depth_before(seg)
        assert d.min() >= 0


def test_grid_boxes_exact():
    k, b = gen.walk(20000, 256, 4, gen.BOX_GRID)
    rows = np.isin(k, [0, 1])
    assert (np.floor(b[rows] * 256) == b[rows] * 256).all()
    assert (b[rows, 2] - b[rows, 0] >= 2.0 ** -8).all()


def test_interleave_keeps_tree_order_and_is_seeded():
    kind, box = gen.walk(500, 8, 31)
    tag, sbox, pos = gen.interleave(kind, box, 2000, 32)
    assert pos.shape == (500,) and np.all(np.diff(pos) > 0)
    assert np.array_equal(tag[pos], kind) and np.array_equal(sbox[pos], box)
    assert (np.delete(tag, pos) == gen.OTHER).all() and np.isfinite(sbox).all()
    t2, b2, p2 = gen.interleave(kind, box, 2000, 32)
    assert np.array_equal(t2, tag) and np.array_equal(b2, sbox)
    t3, _, _ = gen.interleave(kind, box, 2000, 33)
    assert not np.array_equal(t3, tag)
    # each position is taken with probability m/n
    hits = np.zeros(40)
    k4 = np.zeros(10, np.uint32)
    for s in range(2000):
        t, _, _ = gen.interleave(k4, np.zeros((10, 4), np.float32), 40, 1000 + s)
        hits += t != gen.OTHER
    assert np.all(np.abs(hits / 2000 - 0.25) < 0.05)
    # m == n and m == 0
    t, _, p = gen.interleave(kind, box, 500, 34)
    assert np.array_equal(t, kind)
    t, _, p = gen.interleave(kind[:0], box[:0], 50, 35)
    assert (t == gen.OTHER).all() and p.shape == (0,)
