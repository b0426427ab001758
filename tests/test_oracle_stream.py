"""Pins of the oracle's draw-object stream front end (no GPU).

The front end extracts the tree's elements from a stream that also holds
elements outside the tree (tag 5), runs the walk on the extracted sequence
and puts every result back at its stream position (Introduction: the
renderer runs the algorithm only on the nodes a stream compaction
extracts).  The brute-force definitions of clips (path to the root) and
blends (union over the open..close slice) are stated on the raw stream,
where a tag-5 element is neither a leaf nor a clip nor a bracket, so they
pin the compaction, the walk and the translation back without compacting
anything.
"""
import numpy as np
import pytest

import brute
import gen
import oracle
from test_oracle import _nested_boxes, _well_nested

OTHER = 5


def _check_vs_brute(tag, box):
    m, out, st = oracle.bbox_stream(tag, box)
    assert st == 0
    _, bm, bout = brute.boxes(tag, box)
    tree = tag <= 4
    assert np.array_equal(m[tree], bm[tree])
    assert np.array_equal(out[tree].view(np.uint32), bout[tree].view(np.uint32))
    # positions outside the tree are not written
    assert (m[~tree] == -7).all() and np.isnan(out[~tree]).all()
    return m, out


def test_exhaustive_small_streams():
    rng = np.random.default_rng(11)
    count = 0
    for L in range(0, 8):
        for seq in _well_nested(L):
            kind = np.array(seq, np.uint32)
            box = _nested_boxes(kind, rng)
            n = L + int(rng.integers(0, 2 * L + 2))
            tag, sbox, pos = gen.interleave(kind, box, n, 500 + count)
            _check_vs_brute(tag, sbox)
            count += 1
    # sum over L of sum_k C(L, 2k) Catalan(k) 2^k: every well-nested sequence
    assert count == 888


@pytest.mark.parametrize("seed", range(6))
def test_stream_vs_brute_random(seed):
    m_tree = [40, 200, 700, 1200, 300, 40][seed]
    dens = [0.1, 0.25, 0.5, 0.9, 1.0, 0.02][seed]
    kind, box = gen.walk(m_tree, [3, 8, 64, 500, 16, 4][seed], 3000 + seed, gen.BOX_NESTED_ALL)
    n = int(round(m_tree / dens))
    tag, sbox, pos = gen.interleave(kind, box, n, 3100 + seed)
    m, out = _check_vs_brute(tag, sbox)
    assert (out[pos][:, 0] < out[pos][:, 2]).sum() > 0  # non-trivial boxes


def test_without_other_elements_equals_plain_walk():
    kind, box = gen.walk(4000, 64, 21, gen.BOX_INDEP)
    m, out, st = oracle.bbox_stream(kind, box)
    m0, _, out0, st0 = oracle.bbox(kind, box)
    assert st == st0 == 0
    assert np.array_equal(m, m0) and np.array_equal(out.view(np.uint32), out0.view(np.uint32))


def test_results_do_not_depend_on_placement():
    kind, box = gen.walk(3000, 32, 22, gen.BOX_INDEP)
    rows, partners = [], []
    for s in range(3):
        tag, sbox, pos = gen.interleave(kind, box, 3000 * (s + 2), 40 + s)
        m, out, st = oracle.bbox_stream(tag, sbox)
        assert st == 0
        rows.append(out[pos].view(np.uint32))
        inv = np.full(tag.shape[0], -1, np.int64)
        inv[pos] = np.arange(pos.shape[0])
        partners.append(np.where(m[pos] >= 0, inv[np.maximum(m[pos], 0)], -1))
    for r, p in zip(rows[1:], partners[1:]):
        assert np.array_equal(r, rows[0]) and np.array_equal(p, partners[0])


def test_only_other_elements_and_empty():
    tag = np.full(100, OTHER, np.uint32)
    box = np.ones((100, 4), np.float32)
    m, out, st = oracle.bbox_stream(tag, box)
    assert st == 0 and (m == -7).all() and np.isnan(out).all()
    m, out, st = oracle.bbox_stream(np.zeros(0, np.uint32), np.zeros((0, 4), np.float32))
    assert st == 0 and m.shape == (0,)


def test_status_bits():
    z = lambda n: np.zeros((n, 4), np.float32)
    # tags above 5: BAD_KIND, and dropped like tag 5
    kind, box = gen.walk(200, 8, 23, gen.BOX_INDEP)
    tag, sbox, pos = gen.interleave(kind, box, 500, 24)
    bad = tag.copy()
    bad[tag == OTHER] = np.array([6, 7, 0xFFFFFFFF], np.uint32)[np.arange((tag == OTHER).sum()) % 3]
    m1, o1, st1 = oracle.bbox_stream(bad, sbox)
    m0, o0, st0 = oracle.bbox_stream(tag, sbox)
    assert st0 == 0 and st1 == oracle.BAD_KIND
    assert np.array_equal(m1[pos], m0[pos]) and np.array_equal(o1[pos].view(np.uint32),
                                                               o0[pos].view(np.uint32))
    # unbalanced and mismatched brackets across tag-5 gaps
    t = np.array([1, 5, 5, 2, 5, 2], np.uint32)
    assert oracle.bbox_stream(t, z(6))[2] & oracle.UNBALANCED
    t = np.array([5, 1, 5, 4, 5], np.uint32)
    assert oracle.bbox_stream(t, z(5))[2] == oracle.KIND_MISMATCH
    t = np.array([3, 5, 5], np.uint32)
    assert oracle.bbox_stream(t, z(3))[2] == oracle.UNBALANCED
