"""Pins of the oracle's reference gradient (no GPU).

The gradient rule is this project's own (the paper has no backward pass):
each output coordinate routes to the lowest-index input coordinate that
attains it, and sums are exact 64-bit fixed point (2^-32 grid) rounded once
to fp32.  Pinned here by (a) fp64 central finite differences against the
exact rational gradient on tie-free coordinates, (b) exact integer sums done
independently with Python integers, (c) a brute-force router written from
the rule over the brute-force tree structures, (d) the all-leaf closed form.
"""
from fractions import Fraction

import numpy as np
import pytest

import brute
import gen
import oracle


def rne_f32_of_int(v):
    """Round an exact Python integer to the nearest fp32 (ties to even)."""
    s = -1 if v < 0 else 1
    a = abs(v)
    e = a.bit_length() - 24
    if e > 0:
        q, r = divmod(a, 1 << e)
        half = 1 << (e - 1)
        if r > half or (r == half and (q & 1)):
            q += 1
        a = q << e
    return np.float32(s * a)


def q32(g):
    return round(Fraction(float(g)) * (1 << 32))  # Python round: half to even


def brute_sources(kind, box):
    pm, m, out = brute.boxes(kind, box)
    n = len(kind)
    src = np.full((n, 4), -1, np.int64)
    nonempty = (out[:, 0] < out[:, 2]) & (out[:, 1] < out[:, 3])
    for o in range(n):
        if kind[o] in (brute.LEAF, brute.BCLIP) and nonempty[o]:
            anc = []
            a = pm[o]
            while a >= 0:
                if kind[a] == brute.BCLIP:
                    anc.append(a)
                a = pm[a]
            for c in range(4):
                cand = [e for e in [o] + anc if box[e, c] == out[o, c]]
                src[o, c] = min(cand)
    for o in range(n):
        if kind[o] == brute.ECLIP:
            src[o] = src[m[o]]
    for o in range(n):
        if kind[o] == brute.EBLEND and nonempty[o]:
            op = m[o]
            for c in range(4):
                cand = [src[l, c] for l in range(op + 1, o)
                        if kind[l] == brute.LEAF and nonempty[l] and out[l, c] == out[o, c]]
                src[o, c] = src[op, c] = min(cand)
    return src, out


def tied_case(n, seed):
    """Boxes nested inside their clip ancestor on a coarse grid, so that
    intersections are non-empty and ties between levels are frequent."""
    kind, _ = gen.walk(n, 12, seed, gen.BOX_GRID)
    rng = np.random.default_rng(seed)
    box = np.zeros((n, 4), np.float32)
    stack = []
    for i, k in enumerate(kind):
        if k in (0, 1):
            a = box[stack[-1]] if stack else np.array([0, 0, 64, 64], np.float32)
            x0 = a[0] + 8 * rng.integers(-1, 3)
            y0 = a[1] + 8 * rng.integers(-1, 3)
            box[i] = [x0, y0, x0 + 8 * rng.integers(1, 8), y0 + 8 * rng.integers(1, 8)]
        if k == 1:
            stack.append(i)
        elif k == 2:
            stack.pop()
    return kind, box


@pytest.mark.parametrize("seed", range(6))
def test_sources_vs_brute_router(seed):
    kind, box = tied_case([40, 200, 700][seed % 3], 300 + seed)
    src, st = oracle.sources(kind, box)
    assert st == 0
    bsrc, out = brute_sources(kind, box)
    assert np.array_equal(src, bsrc)
    assert (src >= 0).mean() > 0.2
    # ties really occur: some clip-ancestor coordinate equals a leaf's own one
    ties = sum(1 for o in range(len(kind)) for c in range(4)
               if kind[o] == 0 and 0 <= src[o, c] < o)
    assert ties > 0


@pytest.mark.parametrize("seed", range(4))
def test_exact_fixed_point_accumulation(seed):
    kind, box = tied_case(600, 400 + seed)
    n = len(kind)
    g = gen.normal(4 * n, 500 + seed).reshape(n, 4)
    g[::5] *= np.float32(1e-6)  # small values exercise the grid rounding
    gi, st = oracle.backward(kind, box, g)
    assert st == 0
    src, _ = brute_sources(kind, box)
    acc = {}
    for o in range(n):
        for c in range(4):
            if src[o, c] >= 0:
                key = (int(src[o, c]), c)
                acc[key] = acc.get(key, 0) + q32(g[o, c])
    want = np.zeros((n, 4), np.float32)
    for (e, c), v in acc.items():
        want[e, c] = rne_f32_of_int(v) * np.float32(2.0 ** -32)
    assert np.array_equal(gi.view(np.uint32), want.view(np.uint32))


def test_all_leaves_closed_form():
    n = 500
    kind = np.zeros(n, np.uint32)
    _, box = gen.walk(n, 0, 7, gen.BOX_GRID)
    g = gen.normal(4 * n, 8).reshape(n, 4)
    gi, st = oracle.backward(kind, box, g)
    assert st == 0
    want = np.array([[rne_f32_of_int(q32(v)) * np.float32(2.0 ** -32) for v in row] for row in g],
                    np.float32)
    assert np.array_equal(gi, want)


def _fd_case(n, seed):
    kind, box = gen.walk(n, 256, seed, gen.BOX_GRID)
    # nest the grid boxes so clips and unions attain from many places
    rng = np.random.default_rng(seed)
    stack = []
    for i, k in enumerate(kind):
        if k in (0, 1) and stack and rng.random() < 0.9:
            a = box[stack[-1]]
            w = box[i, 2] - box[i, 0]
            h = box[i, 3] - box[i, 1]
            box[i, 0] = a[0] + np.float32(np.floor(rng.random() * 256) / 256 * 64)
            box[i, 1] = a[1] + np.float32(np.floor(rng.random() * 256) / 256 * 64)
            box[i, 2] = box[i, 0] + w
            box[i, 3] = box[i, 1] + h
        if k == 1:
            stack.append(i)
        elif k == 2:
            stack.pop()
    return kind, box


def test_finite_differences_fp64():
    """Central differences (h = 2^-10, grid step 2^-8) of the fp64 walk match
    the exact (rational) gradient to 1e-9 relative on 512 tie-free coordinates."""
    kind, box = _fd_case(3000, 11)
    n = len(kind)
    g = gen.normal(4 * n, 12).reshape(n, 4)
    src, st = oracle.sources(kind, box)
    assert st == 0
    base, _ = oracle.bbox_f64(kind, box.astype(np.float64))
    rng = np.random.default_rng(13)
    rows = np.nonzero(np.isin(kind, [0, 1]))[0]
    h = 2.0 ** -10
    done, tried, nonzero = 0, 0, 0
    g64 = g.astype(np.float64)
    routed = sorted({(int(v), cc) for (o, cc), v in np.ndenumerate(src) if v >= 0})
    while done < 512:
        tried += 1
        assert tried < 20000
        if rng.random() < 0.8:  # mostly coordinates that some output attains
            e, c = routed[int(rng.integers(0, len(routed)))]
        else:
            e, c = int(rng.choice(rows)), int(rng.integers(0, 4))
        outs = {}
        for step in (h, -h, h / 2, -h / 2):
            b = box.astype(np.float64)
            b[e, c] += step
            outs[step], _ = oracle.bbox_f64(kind, b)
        with np.errstate(invalid="ignore"):
            d1 = outs[h] - base
            d2 = base - outs[-h]
            d3 = outs[h / 2] - base
        fin = np.isfinite(base)
        if not (np.array_equal(np.isfinite(outs[h]), fin) and np.array_equal(np.isfinite(outs[-h]), fin)):
            continue  # a box switched between EMPTY and non-EMPTY: not differentiable here
        d1, d2, d3 = d1[fin], d2[fin], d3[fin]
        if not (np.array_equal(d1, d2) and np.array_equal(d1, 2 * d3)
                and np.isin(d1, [0.0, h, -h]).all()):
            continue  # a tie: one-sided derivatives differ
        fd = float(np.sum(g64[fin] * (outs[h][fin] - outs[-h][fin]))) / (2 * h)
        exact = sum(Fraction(float(g[o, cc])) for o, cc in zip(*np.nonzero(src == e))
                    if cc == c)
        exact = float(exact)
        if exact == 0.0:
            assert abs(fd) <= 1e-12
        else:
            nonzero += 1
            assert abs(fd - exact) <= 1e-9 * abs(exact), (e, c, fd, exact)
        done += 1
    assert nonzero > 100


def _clip_over_leaves(m):
    """One BEGIN_CLIP (0,0,10,10) over m leaves that each stick out on every
    side, so every coordinate of every row is attained by the clip alone."""
    kind = np.array([1] + [0] * m + [2], np.uint32)
    box = np.zeros((m + 2, 4), np.float32)
    box[0] = [0, 0, 10, 10]
    box[1:m + 1] = [-5, -5, 20, 20]
    return kind, box


def test_tiny_contributions_on_the_grid():
    """The rule rounds each g to the 2^-32 grid before summing: several
    |g| < 2^-9 contributions landing on one coordinate give RNE(sum of
    q32(g)), which is not the correctly rounded exact sum (the reading of
    the gradient rule: an int64 grid, not the 2^-64 / int128 one)."""
    m = 9
    kind, box = _clip_over_leaves(m)
    tiny = np.array([3e-10, -7e-11, 1.5e-9, 2.0 ** -33, -(2.0 ** -33), 1.5 * 2.0 ** -33,
                     2.5 * 2.0 ** -33, 1e-12, 2.0 ** -10], np.float32)
    g = np.zeros((m + 2, 4), np.float32)
    for c in range(4):
        g[1:m + 1, c] = np.roll(tiny, c) * (1 if c % 2 == 0 else -1)
    g[0] = [2.0 ** -20, 0.0, 0.0, 0.0]  # the clip's own row routes to itself
    g[m + 1] = [0.0, 3e-11, 0.0, -(2.0 ** -12)]  # END_CLIP routes like its BEGIN_CLIP
    gi, st = oracle.backward(kind, box, g)
    assert st == 0
    inexact = 0
    for c in range(4):
        contribs = [g[o, c] for o in range(m + 2)]
        want = rne_f32_of_int(sum(q32(v) for v in contribs)) * np.float32(2.0 ** -32)
        assert gi[0, c].view(np.uint32) == np.float32(want).view(np.uint32), (c, gi[0, c], want)
        exact = np.float32(float(sum(Fraction(float(v)) for v in contribs)))
        inexact += int(exact != gi[0, c])
    assert inexact >= 2  # the grid rounding really shows
    assert (gi[1:] == 0).all()
    # 2^-33 itself rounds to 0 (half to even); 1.5 * 2^-33 and 2.5 * 2^-33 to 2^-32
    assert q32(np.float32(2.0 ** -33)) == 0 and q32(np.float32(1.5 * 2.0 ** -33)) == 1
    assert q32(np.float32(2.5 * 2.0 ** -33)) == 1


def test_grad_range_status():
    """A routed |g| >= 2^31 (or NaN) has no q32 and sets GRAD_RANGE (16); a
    NaN on a coordinate that routes nothing is ignored."""
    kind, box = _clip_over_leaves(3)
    g = np.ones((5, 4), np.float32)
    g[2, 1] = np.float32(3e9)
    _, st = oracle.backward(kind, box, g)
    assert st == 16
    g[2, 1] = np.nan
    _, st = oracle.backward(kind, box, g)
    assert st == 16
    g[2, 1] = np.float32(2.0 ** 31 - 128)  # the largest fp32 below 2^31 is fine
    _, st = oracle.backward(kind, box, g)
    assert st == 0
    kind2 = np.array([1, 0, 2], np.uint32)
    box2 = np.array([[0, 0, 10, 10], [20, 20, 30, 30], [0, 0, 0, 0]], np.float32)  # leaf clipped EMPTY
    g2 = np.ones((3, 4), np.float32)
    g2[1] = np.nan
    _, st = oracle.backward(kind2, box2, g2)
    assert st == 0


def test_finite_differences_on_the_16m_gradient_scene():
    """The FP64 central-difference check on 512 coordinates of the 2^24
    gradient scene itself (cap 256, 2^-8 grid, N(0,1) upstream gradient),
    against the exact rational gradient that the oracle's routing gives, to
    1e-9 relative.  A perturbation of one input coordinate changes only rows
    of the top-level subtree holding it (the root context is the whole
    plane and no union crosses depth 0), so each central difference runs
    the fp64 walk on that subtree alone; coordinates are drawn by seed from
    those whose subtree has at most 2^20 elements, and, as in the smaller
    check, ties (one-sided derivatives that differ) are redrawn."""
    c = gen.config(4)
    kind, box, g = c["kind"], c["box"], c["grad"]
    n = len(kind)
    src, st = oracle.sources(kind, box)
    assert st == 0
    depth = np.cumsum(np.where(np.isin(kind, (1, 3)), 1, np.where(np.isin(kind, (2, 4)), -1, 0)))
    starts = np.concatenate([[0], np.flatnonzero(depth[:-1] == 0) + 1])  # top-level subtrees
    seg_of = np.searchsorted(starts, np.arange(n), side="right") - 1
    seg_end = np.append(starts[1:], n)
    flat = src.reshape(-1)
    routed = np.flatnonzero(flat >= 0)
    order = routed[np.argsort(flat[routed] * 4 + routed % 4, kind="stable")]  # by (source, coordinate)
    keys = flat[order] * 4 + order % 4
    h = 2.0 ** -10
    rng = np.random.default_rng(0x4FD)
    cand = np.unique(keys)
    done = nonzero = tried = 0
    while done < 512:
        tried += 1
        assert tried < 20000
        key = int(cand[int(rng.integers(0, len(cand)))])
        e, cc = divmod(key, 4)
        a, b = int(starts[seg_of[e]]), int(seg_end[seg_of[e]])
        if b - a > (1 << 20):
            continue
        kk, bb = kind[a:b], box[a:b].astype(np.float64)
        base, _ = oracle.bbox_f64(kk, bb)
        outs = {}
        for step in (h, -h, h / 2, -h / 2):
            b2 = bb.copy()
            b2[e - a, cc] += step
            outs[step], _ = oracle.bbox_f64(kk, b2)
        fin = np.isfinite(base)
        if not (np.array_equal(np.isfinite(outs[h]), fin) and np.array_equal(np.isfinite(outs[-h]), fin)):
            continue
        with np.errstate(invalid="ignore"):
            d1, d2, d3 = (outs[h] - base)[fin], (base - outs[-h])[fin], (outs[h / 2] - base)[fin]
        if not (np.array_equal(d1, d2) and np.array_equal(d1, 2 * d3) and np.isin(d1, [0.0, h, -h]).all()):
            continue  # a tie
        fd = float(np.sum(g[a:b].astype(np.float64)[fin] * (outs[h][fin] - outs[-h][fin]))) / (2 * h)
        lo, hi = np.searchsorted(keys, key), np.searchsorted(keys, key, side="right")
        exact = float(sum(Fraction(float(g.reshape(-1)[r])) for r in order[lo:hi]))
        if exact == 0.0:
            assert abs(fd) <= 1e-12
        else:
            nonzero += 1
            assert abs(fd - exact) <= 1e-9 * abs(exact), (e, cc, fd, exact)
        done += 1
    assert nonzero > 400
