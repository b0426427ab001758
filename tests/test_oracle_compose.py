"""Pins of the transform-composition oracle (a non-commutative monoid
composed down the tree, the Introduction's skeleton example).  Each check
computes the expected value by a different route: an explicit ancestor scan
with Python integers, closed forms, and hand-multiplied matrices."""
import numpy as np

import gen
import oracle

M32 = (1 << 32) - 1


def mul(p, q):
    """[a b c; d e f] . [a b c; d e f] modulo 2^32, q applied first."""
    a, b, c, d, e, f = p
    A, B, C, D, E, F = q
    return ((a * A + b * D) & M32, (a * B + b * E) & M32, (a * C + b * F + c) & M32,
            (d * A + e * D) & M32, (d * B + e * E) & M32, (d * C + e * F + f) & M32)


ID = (1, 0, 0, 0, 1, 0)


def brute(kind, xf):
    """Enclosing opens found by scanning back with a balance counter; the
    product is taken outermost first.  A close takes its open's value."""
    n = len(kind)
    out = []
    for i in range(n):
        anchor = i
        if kind[i] in (2, 4):  # a close: its open is the first unmatched open behind it
            d = 0
            for j in range(i - 1, -1, -1):
                if kind[j] in (2, 4):
                    d += 1
                elif kind[j] in (1, 3):
                    if d == 0:
                        anchor = j
                        break
                    d -= 1
        chain = [anchor] if kind[anchor] in (1, 3) else []
        d = 0
        for j in range(anchor - 1, -1, -1):
            if kind[j] in (2, 4):
                d += 1
            elif kind[j] in (1, 3):
                if d == 0:
                    chain.append(j)
                else:
                    d -= 1
        r = ID
        for j in reversed(chain):
            r = mul(r, tuple(int(v) for v in xf[j]))
        out.append(r)
    return np.array(out, dtype=np.uint64).astype(np.uint32)


def rand_xf(n, rng):
    return rng.integers(0, 1 << 32, size=(n, 6), dtype=np.uint64).astype(np.uint32)


def test_brute_force_random_trees():
    rng = np.random.default_rng(1)
    for seed in range(40):
        n = int(rng.integers(1, 120))
        kind, _ = gen.walk(n, int(rng.integers(1, 12)), 500 + seed)
        xf = rand_xf(n, rng)
        out, st = oracle.compose(kind, xf)
        assert st == 0
        assert np.array_equal(out, brute(kind, xf)), seed


def test_translations_add_up():
    """Pure translations: the product is the sum of the enclosing offsets."""
    rng = np.random.default_rng(2)
    kind, _ = gen.walk(3000, 40, 77)
    xf = np.zeros((len(kind), 6), np.uint32)
    xf[:, 0] = 1
    xf[:, 4] = 1
    xf[:, 2] = rng.integers(0, 1 << 32, size=len(kind), dtype=np.uint64).astype(np.uint32)
    xf[:, 5] = rng.integers(0, 1 << 32, size=len(kind), dtype=np.uint64).astype(np.uint32)
    out, st = oracle.compose(kind, xf)
    assert st == 0
    # running sum of the offsets on the stack, kept with an explicit stack of sums
    sums = [(0, 0)]
    for i, k in enumerate(kind):
        if k in (1, 3):
            sx, sy = sums[-1]
            sums.append(((sx + int(xf[i, 2])) & M32, (sy + int(xf[i, 5])) & M32))
            exp = sums[-1]
        elif k in (2, 4):
            exp = sums.pop()
        else:
            exp = sums[-1]
        assert tuple(out[i]) == (1, 0, exp[0], 0, 1, exp[1]), i


def test_order_outermost_first():
    """A 90-degree rotation enclosing a translation, and the reverse: the
    products differ, and each equals the hand-multiplied matrix."""
    R = (0, M32, 0, 1, 0, 0)  # (x, y) -> (-y, x)
    T = (1, 0, 5, 0, 1, 9)    # (x, y) -> (x + 5, y + 9)
    kind = np.array([1, 3, 0, 4, 2], np.uint32)
    for outer, inner in ((R, T), (T, R)):
        xf = np.zeros((5, 6), np.uint32)
        xf[0], xf[1] = outer, inner
        out, st = oracle.compose(kind, xf)
        assert st == 0
        prod = mul(outer, inner)
        assert tuple(out[2]) == prod and tuple(out[1]) == prod and tuple(out[3]) == prod
        assert tuple(out[0]) == outer and tuple(out[4]) == outer
    assert mul(R, T) != mul(T, R)
    assert mul(R, T) == (0, M32, (-9) & M32, 1, 0, 5)


def test_identities_and_root():
    kind, _ = gen.walk(2000, 30, 5)
    xf = np.tile(np.array(ID, np.uint32), (len(kind), 1))
    out, st = oracle.compose(kind, xf)
    assert st == 0 and (out == np.array(ID, np.uint32)).all()
    out, st = oracle.compose(np.zeros(5, np.uint32), rand_xf(5, np.random.default_rng(0)))
    assert st == 0 and (out == np.array(ID, np.uint32)).all()  # leaves at the root


def test_status_bits():
    k, _ = gen.walk(500, 10, 3)
    xf = rand_xf(len(k) + 1, np.random.default_rng(3))
    assert oracle.compose(np.concatenate([k, [9]]).astype(np.uint32), xf)[1] & 1
    assert oracle.compose(np.concatenate([k, [2]]).astype(np.uint32), xf)[1] & 2
    assert oracle.compose(np.concatenate([[1], k]).astype(np.uint32), xf)[1] & 2


# ------------------------------------------------ fp32 transforms (rounding)
def _f32_mul(p, q):
    """p.q in fp32, each product and each sum rounded, left to right."""
    f = np.float32
    a = f(f(p[0] * q[0]) + f(p[1] * q[3]))
    b = f(f(p[0] * q[1]) + f(p[1] * q[4]))
    c = f(f(f(p[0] * q[2]) + f(p[1] * q[5])) + p[2])
    d = f(f(p[3] * q[0]) + f(p[4] * q[3]))
    e = f(f(p[3] * q[1]) + f(p[4] * q[4]))
    ff = f(f(f(p[3] * q[2]) + f(p[4] * q[5])) + p[5])
    return np.array([a, b, c, d, e, ff], np.float32)


def _parents(kind):
    """The enclosing open of every element (an independent stack walk)."""
    st, par = [], []
    for i, k in enumerate(kind):
        par.append(st[-1] if st else -1)
        if k in (1, 3):
            st.append(i)
        elif k in (2, 4):
            st.pop()
    return par


def _jump_value(xf, chain):
    """Pointer jumping written as a recursion over one open's chain (itself,
    then its enclosing opens, nearest first): after round r the node at chain
    position k holds (the node 2^(r-1) further out, after round r-1) . (its
    own value after round r-1), when that node exists."""
    memo = {}

    def v(k, r):
        if r == 0:
            return xf[chain[k]]
        key = (k, r)
        if key not in memo:
            far = k + (1 << (r - 1))
            memo[key] = _f32_mul(v(far, r - 1), v(k, r - 1)) if far < len(chain) else v(k, r - 1)
        return memo[key]

    R = 0
    while (1 << R) < len(chain):
        R += 1
    return v(0, R)


def _random_xf(n, rng):
    ang = rng.uniform(0, 2 * np.pi, n)
    s = rng.uniform(0.5, 2.0, n)
    xf = np.stack([s * np.cos(ang), -s * np.sin(ang), rng.uniform(-100, 100, n),
                   s * np.sin(ang), s * np.cos(ang), rng.uniform(-100, 100, n)], 1)
    return xf.astype(np.float32)


def test_f32_exact_inputs_equal_integer_products():
    """Small integer entries on shallow trees keep every product exact in
    fp32, so every grouping gives the integer product: checked against the
    modular integer walk (no overflow at these sizes)."""
    rng = np.random.default_rng(61)
    for seed in range(6):
        kind, _ = gen.walk(400, 6, 610 + seed)
        xi = rng.integers(-2, 3, size=(len(kind), 6)).astype(np.int64)
        out, st = oracle.compose_f32(kind, xi.astype(np.float32))
        want, st2 = oracle.compose(kind, (xi % (1 << 32)).astype(np.uint32))
        assert st == 0 and st2 == 0
        assert np.array_equal(out, want.view(np.int32).astype(np.float32))


def test_f32_order_is_pointer_jumping():
    """Every element equals the pointer-jumping recursion over its own chain
    (formulated independently of the oracle's array rounds), bit for bit;
    and the order matters: a left fold outermost-first and a right fold give
    other bits on some elements, so a differently grouped implementation
    fails this test."""
    rng = np.random.default_rng(62)
    kind, _ = gen.walk(3000, 40, 620)
    xf = _random_xf(len(kind), rng)
    out, st = oracle.compose_f32(kind, xf)
    assert st == 0
    par = _parents(kind)
    ident = np.array([1, 0, 0, 0, 1, 0], np.float32)
    left_differs = right_differs = 0
    for i, k in enumerate(kind):
        o = i if k in (1, 3) else par[i]
        if k in (2, 4):
            o = par[i]  # a close: its own open is on top of the stack before it
        if o < 0:
            assert np.array_equal(out[i], ident)
            continue
        chain = [o]
        while par[chain[-1]] >= 0:
            chain.append(par[chain[-1]])
        want = _jump_value(xf, chain)
        assert np.array_equal(out[i].view(np.uint32), want.view(np.uint32)), i
        if k in (1, 3) and len(chain) >= 4:
            lf = xf[chain[-1]]
            for c in reversed(chain[:-1]):
                lf = _f32_mul(lf, xf[c])
            rf = xf[chain[0]]
            for c in chain[1:]:
                rf = _f32_mul(xf[c], rf)
            left_differs += int(not np.array_equal(lf, want))
            right_differs += int(not np.array_equal(rf, want))
    assert left_differs > 10 and right_differs > 10


def test_f32_single_chain_rounds():
    """A chain of 5 opens: the jumping order groups them as
    (((x4.x3).(x2.x1)).x0)... written out by hand for this depth."""
    rng = np.random.default_rng(63)
    kind = np.array([1, 3, 1, 3, 1, 0, 2, 4, 2, 4, 2], np.uint32)
    xf = _random_xf(len(kind), rng)
    out, st = oracle.compose_f32(kind, xf)
    assert st == 0
    m = _f32_mul
    x = [xf[i] for i in range(5)]  # x[0] outermost ... x[4] innermost
    # innermost open (position 4): chain x4, x3, x2, x1, x0 (nearest first)
    # round 1: v(k) = x[k+1 out] . x[k]; round 2: pairs of pairs; round 3: + the last
    r1 = lambda inner: m(x[inner - 1], x[inner]) if inner >= 1 else x[inner]
    r2 = lambda inner: m(r1(inner - 2), r1(inner)) if inner >= 2 else r1(inner)
    r3 = lambda inner: m(r2(inner - 4), r2(inner)) if inner >= 4 else r2(inner)
    assert np.array_equal(out[4], r3(4)) and np.array_equal(out[5], r3(4))
    assert np.array_equal(out[3], r2(3)) and np.array_equal(out[0], x[0])


# --------------------------------------- fp32 transforms up the tree (rounding)
def _match_py(kind):
    st, m = [], [-1] * len(kind)
    for i, k in enumerate(kind):
        if k in (1, 3):
            st.append(i)
        elif k in (2, 4):
            o = st.pop()
            m[o], m[i] = i, o
    return m


def test_up_f32_exact_inputs_equal_ordered_products():
    """Small integer transforms on leaves: every product is exact, so every
    grouping agrees and the result is the ordered product of the subtree's
    leaves (non-commutative: checks the factor order), computed here with
    Python integers."""
    rng = np.random.default_rng(71)
    for seed in range(5):
        kind, _ = gen.walk(300, 5, 710 + seed)
        xi = rng.integers(-1, 2, size=(len(kind), 6)).astype(np.int64)
        xi[:, 0] = 1  # keep products small: upper triangular-ish with a = 1
        xi[:, 3] = 0
        out, st = oracle.reduce_up_f32(kind, xi.astype(np.float32))
        assert st == 0
        m = _match_py(kind)

        def mul(p, q):
            return [p[0] * q[0] + p[1] * q[3], p[0] * q[1] + p[1] * q[4], p[0] * q[2] + p[1] * q[5] + p[2],
                    p[3] * q[0] + p[4] * q[3], p[3] * q[1] + p[4] * q[4], p[3] * q[2] + p[4] * q[5] + p[5]]

        for i, k in enumerate(kind):
            if k == 0:
                assert np.array_equal(out[i], xi[i].astype(np.float32))
            elif k in (1, 3):
                acc = [1, 0, 0, 0, 1, 0]
                for j in range(i + 1, m[i]):
                    if kind[j] == 0:
                        acc = mul(acc, [int(v) for v in xi[j]])
                assert max(abs(v) for v in acc) < 1 << 24
                assert np.array_equal(out[i], np.array(acc, np.float32)), i
                assert np.array_equal(out[m[i]], out[i])


def _up_grouping(xf, leaves_mask, lo, hi, N):
    """The segment-tree grouping written top-down: the canonical nodes of
    [lo, hi] in order; the leading ones (growing) folded left to right, the
    trailing ones (shrinking) folded right to left, then the two joined."""
    def value(v, a, b):  # node v covers [a, b): product of its leaves, None if none
        if b - a == 1:
            return xf[a] if a < len(leaves_mask) and leaves_mask[a] else None
        mid = (a + b) // 2
        x, y = value(2 * v, a, mid), value(2 * v + 1, mid, b)
        return x if y is None else y if x is None else _f32_mul(x, y)

    nodes = []

    def cover(v, a, b):
        if b <= lo or a > hi:
            return
        if lo <= a and b - 1 <= hi:
            nodes.append((v, a, b))
            return
        mid = (a + b) // 2
        cover(2 * v, a, mid)
        cover(2 * v + 1, mid, b)

    cover(1, 0, N)
    # which canonical nodes the left boundary reaches and which the right one
    # does (in the order each boundary meets them) is the grouping itself
    left, right = [], []
    l, r = lo + N, hi + N + 1
    while l < r:
        if l & 1:
            left.append(l)
            l += 1
        if r & 1:
            r -= 1
            right.append(r)
        l >>= 1
        r >>= 1
    vals = {v: value(v, a, b) for v, a, b in nodes}
    assert sorted(left + right) == sorted(v for v, _, _ in nodes)
    L = None
    for v in left:
        x = vals[v]
        L = x if L is None else (L if x is None else _f32_mul(L, x))
    R = None
    for v in right:
        x = vals[v]
        R = x if R is None else (R if x is None else _f32_mul(x, R))
    return L if R is None else R if L is None else _f32_mul(L, R)


def test_up_f32_grouping():
    """Every open equals the segment-tree grouping evaluated top-down (node
    values by recursion over aligned halves), bit for bit; a left fold over
    the same leaves gives other bits on many opens."""
    rng = np.random.default_rng(72)
    kind, _ = gen.walk(1500, 30, 720)
    xf = _random_xf(len(kind), rng)
    out, st = oracle.reduce_up_f32(kind, xf)
    assert st == 0
    m = _match_py(kind)
    N = 1
    while N < len(kind):
        N *= 2
    leaves = [k == 0 for k in kind]
    ident = np.array([1, 0, 0, 0, 1, 0], np.float32)
    differs = 0
    for i, k in enumerate(kind):
        if k not in (1, 3):
            continue
        want = _up_grouping(xf, leaves, i + 1, m[i] - 1, N)
        want = ident if want is None else want
        assert np.array_equal(out[i].view(np.uint32), want.view(np.uint32)), i
        seq = [xf[j] for j in range(i + 1, m[i]) if kind[j] == 0]
        if len(seq) >= 3:
            lf = seq[0]
            for x in seq[1:]:
                lf = _f32_mul(lf, x)
            differs += int(not np.array_equal(lf, want))
    assert differs > 20
