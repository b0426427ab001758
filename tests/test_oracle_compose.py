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
