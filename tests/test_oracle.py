"""Pins of the CPU oracle (no GPU).

The oracle is the paper's sequential stack walk; these tests check it against
things other than itself: the paper's worked examples (tests/golden), the
algebraic definitions of matching via the bicyclic semigroup and the stack
monoid, brute-force clip and blend definitions, exhaustive enumeration of
small trees, closed-form special cases and invariants.
"""
import itertools
import os

import numpy as np
import pytest

import brute
import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def kinds_from_string(s, clip=True):
    m = {"(": brute.BCLIP if clip else brute.BBLEND, ")": brute.ECLIP if clip else brute.EBLEND,
         ".": brute.LEAF}
    return np.array([m[c] for c in s], np.uint32)


# ----------------------------------------------------------- paper examples
def test_bicyclic_worked_example():
    for row in _read("bicyclic_examples.txt"):
        if row[0] == "bic":
            assert brute.bic(row[1]) == (int(row[2]), int(row[3]))
        elif row[0] == "enum":
            want = [(int(p.split(":")[0]), p.split(":")[1]) for p in row[2:]]
            assert brute.enum(row[1]) == want


def test_stack_slice_worked_example():
    g = {r[0]: r[1:] for r in _read("stack_slice_example.txt")}
    s = g["string"][0]
    want_scan = [tuple(int(v) for v in p.split(",")) for p in g["reverse_scan"]]
    scan = [brute.bic(s[i:]) for i in range(len(s))]  # inclusive reverse scan
    assert scan == want_scan
    total = brute.bic(s)
    pred = [i for i in range(len(s)) if s[i] == "(" and brute.bic(s[i + 1:])[0] == 0]
    assert pred == [int(v) for v in g["predicate_true"]]
    slots = {i: total[1] - brute.bic(s[i:])[1] for i in pred}
    assert slots == {int(p.split(":")[0]): int(p.split(":")[1]) for p in g["slots"]}
    # the compacted slice is exactly the stack monoid's list of unmatched opens
    a, l = brute.stk(brute.enum(s))
    assert (a, l) == (total[0], [i for i, _ in sorted(slots.items(), key=lambda kv: kv[1])])


def test_binary_search_worked_example():
    g = {r[0]: r[1:] for r in _read("fig2_search_example.txt")}
    s, i1 = g["string"][0], int(g["i1"][0])
    final = min(i for i in range(i1 + 1) if brute.bic(s[i:i1])[1] == 0)
    assert final == int(g["final_i"][0])
    assert brute.bic(s[final - 1:i1])[1] == 1
    kind = kinds_from_string(s)
    m, pm, st = oracle.match(kind)
    assert pm[i1] == int(g["match"][0]) == final - 1
    assert st == oracle.UNBALANCED  # the example string leaves two opens unclosed


# ------------------------------------------------------------- algebra laws
def test_bicyclic_monoid_laws():
    vals = [(a, b) for a in range(4) for b in range(4)]
    for x in vals:
        assert brute.bic_op(x, (0, 0)) == x == brute.bic_op((0, 0), x)
    for x, y, z in itertools.product(vals, repeat=3):
        assert brute.bic_op(brute.bic_op(x, y), z) == brute.bic_op(x, brute.bic_op(y, z))


def test_bicyclic_closed_form():
    # Bic(s) = (-min(0, min prefix depth), final depth - min(0, min prefix depth))
    rng = np.random.default_rng(1)
    for _ in range(300):
        s = "".join(rng.choice(list("()."), size=rng.integers(0, 30)))
        d, lo = 0, 0
        for ch in s:
            d += 1 if ch == "(" else (-1 if ch == ")" else 0)
            lo = min(lo, d)
        assert brute.bic(s) == (-lo, d - lo)


def test_stack_monoid_laws_and_homomorphism():
    rng = np.random.default_rng(2)

    def rnd():
        return (int(rng.integers(0, 4)), [int(v) for v in rng.integers(0, 99, rng.integers(0, 4))])

    for _ in range(500):
        x, y, z = rnd(), rnd(), rnd()
        assert brute.stk_op(brute.stk_op(x, y), z) == brute.stk_op(x, brute.stk_op(y, z))
        assert brute.stk_op(x, (0, [])) == x == brute.stk_op((0, []), x)
        # forgetting the values maps Stk onto Bic
        xy = brute.stk_op(x, y)
        assert (xy[0], len(xy[1])) == brute.bic_op((x[0], len(x[1])), (y[0], len(y[1])))


def test_suffix_relation():
    # rev(Stk(enum(s)[i0..i2]))[k] == rev(Stk(enum(s)[i0..i1]))[k+j] when Bic(s[i1..i2]) = (j, 0)
    rng = np.random.default_rng(3)
    hits = 0
    for _ in range(400):
        s = "".join(rng.choice(list("(()).."), size=24))
        e = brute.enum(s)
        i0, i1, i2 = sorted(rng.integers(0, 25, 3))
        j, b = brute.bic(s[i1:i2])
        if b != 0:
            continue
        full = brute.stk(e[i0:i2])[1][::-1]
        pre = brute.stk(e[i0:i1])[1][::-1]
        for k in range(len(full)):
            assert full[k] == pre[k + j]
        hits += 1
    assert hits > 50


# ------------------------------------------------------ matching definitions
@pytest.mark.parametrize("seed", range(12))
def test_matching_vs_bic_and_stk_definitions(seed):
    n = [1, 2, 7, 33, 100, 257, 400, 600][seed % 8]
    kind, box = gen.walk(n, [1, 2, 4, 64][seed % 4], 1000 + seed)
    s = "".join(brute.sym(k) for k in kind)
    m, pm, st = oracle.match(kind)
    assert st == 0
    assert np.array_equal(pm, brute.pm_bic(s))
    if n <= 260:
        assert np.array_equal(pm, brute.pm_stk(s))
    assert np.array_equal(m, brute.match_from_pm(kind, pm))
    # pm is the previous strictly smaller depth
    d = brute.depth_before(kind)
    for i in range(n):
        js = [j for j in range(i) if d[j] < d[i]]
        assert pm[i] == (js[-1] if js else -1)


def _well_nested(L):
    """All sequences of length L over leaf / clip pair / blend pair that nest."""
    out = []

    def rec(prefix, stack):
        if len(prefix) + len(stack) > L:
            return
        if len(prefix) == L:
            if not stack:
                out.append(list(prefix))
            return
        rec(prefix + [brute.LEAF], stack)
        for o, c in ((brute.BCLIP, brute.ECLIP), (brute.BBLEND, brute.EBLEND)):
            rec(prefix + [o], stack + [c])
        if stack:
            rec(prefix + [stack[-1]], stack[:-1])

    rec([], [])
    return out


def _nested_boxes(kind, rng):
    """Small integer boxes that often overlap (so clips and unions are non-trivial)."""
    n = len(kind)
    x0 = rng.integers(0, 6, n).astype(np.float32)
    y0 = rng.integers(0, 6, n).astype(np.float32)
    w = rng.integers(1, 6, n).astype(np.float32)
    h = rng.integers(1, 6, n).astype(np.float32)
    b = np.stack([x0, y0, x0 + w, y0 + h], 1)
    b[~np.isin(kind, [brute.LEAF, brute.BCLIP])] = 0
    return b


def test_exhaustive_small_trees():
    rng = np.random.default_rng(4)
    count = 0
    for L in range(0, 10):
        for seq in _well_nested(L):
            kind = np.array(seq, np.uint32)
            box = _nested_boxes(kind, rng)
            m, pm, out, st = oracle.bbox(kind, box)
            assert st == 0
            bpm, bm, bout = brute.boxes(kind, box)
            assert np.array_equal(pm, bpm) and np.array_equal(m, bm)
            assert np.array_equal(out.view(np.uint32), bout.view(np.uint32)), (seq, out, bout)
            count += 1
    assert count == 9306  # all sequences of length 0..9


@pytest.mark.parametrize("seed", range(8))
def test_boxes_vs_brute_random(seed):
    n = [50, 300, 900, 1500][seed % 4]
    kind, box = gen.walk(n, [3, 8, 64, 500][seed % 4], 2000 + seed, gen.BOX_NESTED_ALL)
    m, pm, out, st = oracle.bbox(kind, box)
    assert st == 0
    bpm, bm, bout = brute.boxes(kind, box)
    assert np.array_equal(pm, bpm) and np.array_equal(m, bm)
    assert np.array_equal(out.view(np.uint32), bout.view(np.uint32))
    assert (out[:, 0] < out[:, 2]).sum() > 0  # some values are non-trivial


# ------------------------------------------------------------ special cases
def test_all_leaves():
    rng = np.random.default_rng(5)
    n = 1000
    kind = np.zeros(n, np.uint32)
    box = _nested_boxes(kind, rng)
    box[::7, 2] = box[::7, 0]  # zero-width rows become EMPTY
    m, pm, out, st = oracle.bbox(kind, box)
    assert st == 0 and (m == -1).all() and (pm == -1).all()
    ok = (box[:, 0] < box[:, 2]) & (box[:, 1] < box[:, 3])
    assert np.array_equal(out[ok], box[ok])
    assert np.array_equal(out[~ok], np.tile(brute.EMPTY, ((~ok).sum(), 1)))


def test_single_clip_chain_is_running_extremum():
    rng = np.random.default_rng(6)
    d = 500
    kind = np.array([brute.BCLIP] * d + [brute.ECLIP] * d, np.uint32)
    box = np.zeros((2 * d, 4), np.float32)
    box[:d, 0] = rng.uniform(0, 10, d)
    box[:d, 1] = rng.uniform(0, 10, d)
    box[:d, 2] = rng.uniform(1000, 2000, d)
    box[:d, 3] = rng.uniform(1000, 2000, d)
    m, pm, out, st = oracle.bbox(kind, box)
    assert st == 0
    want = np.stack([np.maximum.accumulate(box[:d, 0]), np.maximum.accumulate(box[:d, 1]),
                     np.minimum.accumulate(box[:d, 2]), np.minimum.accumulate(box[:d, 3])], 1)
    assert np.array_equal(out[:d], want)
    assert np.array_equal(out[d:], want[::-1])  # END_CLIP carries its BEGIN_CLIP's box
    assert np.array_equal(m[:d], np.arange(2 * d - 1, d - 1, -1))


def test_blends_only_is_range_extremum():
    kind, box = gen.walk(3000, 40, 77, gen.BOX_INDEP)
    kind = np.where(kind == brute.BCLIP, brute.BBLEND, kind)
    kind = np.where(kind == brute.ECLIP, brute.EBLEND, kind).astype(np.uint32)
    box[kind != brute.LEAF] = 0
    m, pm, out, st = oracle.bbox(kind, box)
    assert st == 0
    leaf = kind == brute.LEAF
    lo = np.where(leaf[:, None], box, brute.EMPTY)
    for c in np.nonzero(kind == brute.EBLEND)[0]:
        o = m[c]
        seg = lo[o + 1:c]
        want = (np.array([seg[:, 0].min(), seg[:, 1].min(), seg[:, 2].max(), seg[:, 3].max()],
                         np.float32) if len(seg) else brute.EMPTY)
        assert np.array_equal(out[c], want) and np.array_equal(out[o], want)


# --------------------------------------------------------------- invariants
def test_invariants_workload_64k():
    c = gen.config(0, nested_boxes=True)
    kind, box = c["kind"], c["box"]
    m, pm, out, st = oracle.bbox(kind, box)
    assert st == 0
    n = len(kind)
    opens = np.isin(kind, [1, 3])
    closes = np.isin(kind, [2, 4])
    assert (m[kind == 0] == -1).all()
    idx = np.nonzero(opens | closes)[0]
    assert np.array_equal(m[m[idx]], idx)  # involution
    partner = np.array([0, 2, 1, 4, 3], np.uint32)
    assert np.array_equal(kind[m[idx]], partner[kind[idx]])  # kinds pair up
    d = brute.depth_before(kind)
    assert (d >= 0).all()
    # open and close rows of every node carry the same box
    cl = np.nonzero(closes)[0]
    assert np.array_equal(out[cl], out[m[cl]])
    # every non-empty leaf lies inside the box of each enclosing clip and blend
    ne = (out[:, 0] < out[:, 2])
    for i in np.nonzero((kind == 0) & ne)[0][:2000]:
        a = pm[i]
        while a >= 0:
            b = out[a]
            assert b[0] <= out[i, 0] and b[1] <= out[i, 1] and b[2] >= out[i, 2] and b[3] >= out[i, 3]
            a = pm[a]
    # EMPTY rows are canonical
    e = ~ne & np.isin(kind, [0, 1, 2, 3, 4])
    assert np.array_equal(out[e], np.tile(brute.EMPTY, (e.sum(), 1)))


def test_malformed_inputs_status():
    K = lambda s, clip=True: kinds_from_string(s, clip)
    z = lambda n: np.zeros((n, 4), np.float32)
    assert oracle.bbox(K("())"), z(3))[3] & oracle.UNBALANCED
    assert oracle.bbox(K("(()"), z(3))[3] & oracle.UNBALANCED
    k = np.array([1, 4], np.uint32)  # BEGIN_CLIP closed by END_BLEND
    assert oracle.bbox(k, z(2))[3] == oracle.KIND_MISMATCH
    k = np.array([0, 7, 0], np.uint32)
    assert oracle.bbox(k, z(3))[3] == oracle.BAD_KIND
    assert oracle.bbox(np.zeros(0, np.uint32), z(0))[3] == 0


def test_match_only_agrees_with_bbox():
    kind, box = gen.walk(5000, 64, 9, gen.BOX_INDEP)
    m1, pm1, st1 = oracle.match(kind)
    m2, pm2, _, st2 = oracle.bbox(kind, box)
    assert st1 == st2 == 0 and np.array_equal(m1, m2) and np.array_equal(pm1, pm2)


def test_f64_walk_equals_f32_walk_on_f32_inputs():
    kind, box = gen.walk(20000, 64, 10, gen.BOX_NESTED_ALL)
    _, _, out32, _ = oracle.bbox(kind, box)
    out64, st = oracle.bbox_f64(kind, box.astype(np.float64))
    assert st == 0
    assert np.array_equal(out64.astype(np.float32), out32)
    assert np.array_equal(out64, out32.astype(np.float64))
