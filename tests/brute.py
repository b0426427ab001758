"""Brute-force formulations used to pin the oracle.

Each function restates a definition from arXiv 2205.11659 directly, in a form
unrelated to the oracle's sequential stack walk:
  * Bic(s) and the alternate matching definition (section "The bicyclic
    semigroup"): the enclosing-open / matching index of j is the largest i
    with Bic(s[i..j]).b == 1.
  * The stack monoid Stk and last(Stk(enum(s)[..j])) (section "The stack
    monoid").
  * Clip definition (section "Parallel bounding boxes", Clips): a leaf's box
    is its own box intersected with the clip nodes on its path to the root.
  * Blend definition (same section, Blends): the union over the slice of
    descendants between the open and the close.
Slow on purpose (O(n^2) and worse); only for small inputs.
"""
import numpy as np

LEAF, BCLIP, ECLIP, BBLEND, EBLEND = 0, 1, 2, 3, 4
OPENS = (BCLIP, BBLEND)
CLOSES = (ECLIP, EBLEND)
INF = np.float32(np.inf)
EMPTY = np.array([INF, INF, -INF, -INF], np.float32)


def sym(k):
    return "(" if k in OPENS else (")" if k in CLOSES else ".")


def bic_elem(c):
    return (0, 1) if c == "(" else ((1, 0) if c == ")" else (0, 0))


def bic_op(x, y):
    (a, b), (c, d) = x, y
    m = min(b, c)
    return (a + c - m, b + d - m)


def bic(s):
    r = (0, 0)
    for ch in s:
        r = bic_op(r, bic_elem(ch))
    return r


def stk_op(x, y):
    (a0, l0), (a1, l1) = x, y
    return (a0 + a1 - min(len(l0), a1), l0[: max(0, len(l0) - a1)] + l1)


def stk_elem(i, c):
    return (0, [i]) if c == "(" else ((1, []) if c == ")" else (0, []))


def stk(pairs):
    r = (0, [])
    for i, c in pairs:
        r = stk_op(r, stk_elem(i, c))
    return r


def enum(s):
    return list(enumerate(s))


def pm_bic(s):
    """Enclosing-open index per element: max i with Bic(s[i..j]).b == 1, else -1."""
    n = len(s)
    pm = np.full(n, -1, np.int64)
    for j in range(n):
        acc = (0, 0)  # Bic(s[i..j]) for i = j, built leftwards
        for i in range(j - 1, -1, -1):
            acc = bic_op(bic_elem(s[i]), acc)
            if acc[1] == 1:
                pm[j] = i
                break
    return pm


def pm_stk(s):
    """last(Stk(enum(s)[..j])) per element, -1 when the stack is empty."""
    pm = np.full(len(s), -1, np.int64)
    e = enum(s)
    for j in range(len(s)):
        l = stk(e[:j])[1]
        pm[j] = l[-1] if l else -1
    return pm


def match_from_pm(kind, pm):
    m = np.full(len(kind), -1, np.int64)
    for j, k in enumerate(kind):
        if k in CLOSES and pm[j] >= 0:
            m[j] = pm[j]
            m[pm[j]] = j
    return m


def canon(b):
    return b if (b[0] < b[2] and b[1] < b[3]) else EMPTY.copy()


def isect(a, b):
    return np.array([max(a[0], b[0]), max(a[1], b[1]), min(a[2], b[2]), min(a[3], b[3])],
                    np.float32)


def boxes(kind, box):
    """Clip rows by walking each element's ancestor chain; blend rows by
    union over the open..close slice.  Returns out (n, 4) float32."""
    kind = [int(k) for k in kind]
    s = "".join(sym(k) for k in kind)
    pm = pm_bic(s)
    m = match_from_pm(kind, pm)
    n = len(kind)
    out = np.zeros((n, 4), np.float32)
    for i in range(n):
        if kind[i] in (LEAF, BCLIP):
            b = box[i].astype(np.float32).copy()
            a = pm[i]
            while a >= 0:
                if kind[a] == BCLIP:
                    b = isect(b, box[a])
                a = pm[a]
            out[i] = canon(b)
    for c in range(n):
        if kind[c] == ECLIP:
            out[c] = out[m[c]]
        elif kind[c] == EBLEND:
            o = m[c]
            rows = [r for r in range(o + 1, c) if kind[r] == LEAF]
            if rows:
                sub = out[rows]
                u = np.array([sub[:, 0].min(), sub[:, 1].min(), sub[:, 2].max(), sub[:, 3].max()],
                             np.float32)
            else:
                u = EMPTY.copy()
            out[c] = u
            out[o] = u
    return pm, m, out


def depth_before(kind):
    d = np.zeros(len(kind), np.int64)
    cur = 0
    for i, k in enumerate(kind):
        d[i] = cur
        cur += 1 if k in OPENS else (-1 if k in CLOSES else 0)
    return d
