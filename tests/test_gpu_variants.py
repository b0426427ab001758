"""Every launch variant the autotuner can pick is bit-exact against the
oracle, and the tuner leaves correct outputs and records its choice.

A variant changes elements per thread of the main pass (4 or 8) and of
the reduce pass (4 or 8) and close records per thread of the
cross-partition pass (2, 4, 8); results must not depend on it."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import same_bits, say, to_dev

pytestmark = pytest.mark.gpu


def _inputs():
    a = gen.walk(9_999, 64, 0x7A01, gen.BOX_INSET)  # ragged tail, shallow
    b = gen.chain_around_walk(60_000, 90_000, 64, 0x7A02, gen.BOX_INSET_ND)  # deep, cross pairs
    c = gen.walk(300_001, 5000, 0x7A03, gen.BOX_INSET_ND)  # deep random walk
    return [("walk 9999", *a), ("chain 60K around 90K", *b), ("walk 300001 cap 5000", *c)]


@pytest.fixture(autouse=True)
def _clean_table():
    import paper_2205_11659_amd as tb
    tb.tune_clear()
    yield
    tb.tune_clear()


def _bbox(kind, box):
    import torch
    import paper_2205_11659_amd as tb
    out, m, st = tb.tb_bbox(to_dev(kind), to_dev(box))
    torch.cuda.synchronize()
    return m.cpu().numpy(), out.cpu().numpy(), int(st.item())


def test_every_bbox_variant_bit_exact():
    import paper_2205_11659_amd as tb
    cases = [(name, k, b, oracle.bbox(k, b)) for name, k, b in _inputs()]
    for v in tb.candidates(tb.OP_BBOX):
        for name, k, b, (om, _, oout, ost) in cases:
            tb.variant_set(tb.OP_BBOX, len(k), v)
            say(f"[variant] bbox {v} {name}")
            m, out, st = _bbox(k, b)
            assert ost == 0 and st == 0
            assert np.array_equal(m, om), (v, name)
            assert same_bits(out, oout), (v, name)


def test_every_batched_variant_bit_exact():
    import torch
    import paper_2205_11659_amd as tb
    kind, box, off = gen.batch(60, 2.0, 14.0, 2, 500, 0x7A04, gen.BOX_INSET)
    want = [oracle.bbox(kind[a:b], box[a:b]) for a, b in zip(off[:-1], off[1:])]
    for v in tb.candidates(tb.OP_BBOX_BATCHED):
        tb.variant_set(tb.OP_BBOX_BATCHED, len(kind), v)
        say(f"[variant] batched {v}")
        out, m, st = tb.tb_bbox_batched(to_dev(kind), to_dev(box), to_dev(off))
        torch.cuda.synchronize()
        out, m, st = out.cpu().numpy(), m.cpu().numpy(), st.cpu().numpy()
        assert (st == 0).all()
        for s, (a, b) in enumerate(zip(off[:-1], off[1:])):
            om, _, oout, _ = want[s]
            assert np.array_equal(m[a:b], om) and same_bits(out[a:b], oout), (v, s)


def test_every_match_variant_bit_exact():
    import torch
    import paper_2205_11659_amd as tb
    kind, _ = gen.walk(250_003, 3000, 0x7A05)
    om, opm, ost = oracle.match(kind)
    for v in tb.candidates(tb.OP_MATCH):
        tb.variant_set(tb.OP_MATCH, len(kind), v)
        say(f"[variant] match {v}")
        m, pm, st = tb.tb_match(to_dev(kind))
        torch.cuda.synchronize()
        assert int(st.item()) == 0 and ost == 0
        assert np.array_equal(m.cpu().numpy(), om) and np.array_equal(pm.cpu().numpy(), opm), v


def test_tuner_outputs_and_choice(tmp_path):
    import torch
    import paper_2205_11659_amd as tb
    kind, box = gen.chain_around_walk(100_000, 400_000, 64, 0x7A06, gen.BOX_INSET_ND)
    say(f"[variant] tune_bbox n={len(kind)}")
    res, (out, m, st) = tb.tune_bbox(to_dev(kind), to_dev(box), reps=2)
    torch.cuda.synchronize()
    assert tuple(res["variant"]) in tb.candidates(tb.OP_BBOX)
    assert res["ms"] > 0 and res["default_ms"] >= res["ms"]
    assert tb.variant_get(tb.OP_BBOX, len(kind)) == tuple(res["variant"])
    om, _, oout, _ = oracle.bbox(kind, box)
    assert int(st.item()) == 0
    assert np.array_equal(m.cpu().numpy(), om) and same_bits(out.cpu().numpy(), oout)
    # later calls of the same size class use the choice and stay exact
    m2, out2, st2 = _bbox(kind, box)
    assert st2 == 0 and np.array_equal(m2, om) and same_bits(out2, oout)
    path = tmp_path / "tune.txt"
    tb.tune_save(str(path))
    assert f" {tb.OP_BBOX} " in path.read_text()
    kk, _ = gen.walk(200_000, 300, 0x7A07)
    res, (mm, st) = tb.tune_match(to_dev(kk), reps=2)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and np.array_equal(mm.cpu().numpy(), oracle.match(kk)[0])
    assert tuple(res["variant"]) in tb.candidates(tb.OP_MATCH)
    kind, box, off = gen.batch(50, 4.0, 13.0, 2, 300, 0x7A08, gen.BOX_INSET)
    res, (out, m, st) = tb.tune_bbox_batched(to_dev(kind), to_dev(box), to_dev(off), reps=2)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    out, m = out.cpu().numpy(), m.cpu().numpy()
    for a, b in zip(off[:-1], off[1:]):
        om, _, oout, _ = oracle.bbox(kind[a:b], box[a:b])
        assert np.array_equal(m[a:b], om) and same_bits(out[a:b], oout)
