"""Pins of the oracle's typed bracket matching (no GPU).

Token 0 is no bracket, 2t+1 opens type t, 2t+2 closes type t (section "The
parentheses matching problem", Fig. 1, with several kinds of parentheses).
Pinned by (a) a brute-force partner search written from the definition
(depth counting, then the type of the partner), exhaustively over short
token strings; (b) equality with the element-kind walk on tokens 0..4,
where types 0 and 1 are clip and blend; (c) the single-type case against
the bicyclic definition (the partner of an open is the first later position
where the depth returns below it)."""
import itertools

import numpy as np
import pytest

import gen
import oracle

UNBAL, MISMATCH = 2, 4


def brute(tok):
    """Partner by counting depth forward from each open; pm by counting back."""
    n = len(tok)
    opening = [t != 0 and t % 2 == 1 for t in tok]
    closing = [t != 0 and t % 2 == 0 for t in tok]
    match = [-1] * n
    status = 0
    for i in range(n):
        if not opening[i]:
            continue
        d = 0
        for j in range(i + 1, n):
            d += 1 if opening[j] else -1 if closing[j] else 0
            if d < 0:
                match[i], match[j] = j, i
                if tok[j] != tok[i] + 1:
                    status |= MISMATCH
                break
        else:
            status |= UNBAL
    for j in range(n):
        if closing[j] and match[j] < 0:
            status |= UNBAL
    pm = [-1] * n
    for i in range(n):
        d = 0
        for a in range(i - 1, -1, -1):
            d += -1 if opening[a] else 1 if closing[a] else 0
            if opening[a] and d < 0:
                pm[i] = a
                break
    return match, pm, status


def test_exhaustive_short_strings():
    toks = [0, 1, 2, 3, 4, 5, 6]
    count = 0
    for n in range(0, 6):
        for s in itertools.product(toks, repeat=n):
            m, pm, st = oracle.match_brackets(np.array(s, np.uint32))
            bm, bpm, bst = brute(list(s))
            assert st == bst, (s, st, bst)
            if st & UNBAL == 0:
                assert list(m) == bm, s
            assert list(pm) == bpm or st & UNBAL, s
            count += 1
    assert count == sum(7 ** k for k in range(6))


def test_element_kinds_are_two_bracket_types():
    for seed in range(5):
        kind, _ = gen.walk(3000, 40, 100 + seed)
        k2 = kind.copy()
        if seed % 2:
            closes = np.flatnonzero(k2 == 2)
            k2[closes[::7]] = 4  # mistyped closes
        m, pm, st = oracle.match_brackets(k2)
        om, opm, ost = oracle.match(k2)
        assert st == ost and np.array_equal(m, om) and np.array_equal(pm, opm)


def test_single_type_against_depth_definition():
    tok = gen.brackets(5000, 300, 1, 77)
    m, _, st = oracle.match_brackets(tok)
    assert st == 0
    depth = np.cumsum(np.where(tok == 1, 1, np.where(tok == 2, -1, 0)))
    for i in np.flatnonzero(tok == 1)[:400]:
        after = np.flatnonzero(depth[i:] < depth[i])
        assert m[i] == i + after[0]


@pytest.mark.parametrize("ntypes,p_bad", [(1, 0.0), (4, 0.0), (4, 0.01), (1000, 0.0)])
def test_generated_streams(ntypes, p_bad):
    tok = gen.brackets(2000, 50, ntypes, 900 + ntypes, p_bad)
    m, pm, st = oracle.match_brackets(tok)
    bm, bpm, bst = brute([int(t) for t in tok])
    assert st == bst and list(m) == bm and list(pm) == bpm
    assert (st == MISMATCH) == (p_bad > 0)
    opens = np.flatnonzero(tok % 2 == 1)
    assert np.array_equal(m[m[opens]], opens)  # an involution on brackets
