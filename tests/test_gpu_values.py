"""GPU parity on value-rich deep inputs (BOX_INSET boxes: every clip context
and every leaf non-empty, drawn boxes cut by ancestor clips), with minimum
counts, taken from the oracle, of rows whose values travel through the
long-range stages:

- clip contexts carried from at least 33 partitions back, which only the
  later rounds of the pointer jumping over partitions bring in (round r
  reaches 2^r partitions back);
- blend unions that take part of their value from whole union blocks
  strictly between the open's and the close's partitions (the block-level
  sparse table, at each of its levels 0..3);
- gradient routes to a source element in another partition, through blend
  rows and across many partitions.

Each GPU test prints its counts and compares every row bit for bit with the
oracle.  The same counts are asserted on the CPU by test_inputs_* below, so
a generator change that drains the values fails without a GPU.
"""
import numpy as np
import pytest

import coverage as cv
import gen
import oracle
from gpu_util import gpu_bbox, gpu_batched, same_bits, say, to_dev


def deep_scene():
    """Chains of alternating clip/blend opens around random walks,
    concatenated (6.28M elements): 800,000 opens around 1.3M elements (owner
    links reach back 781 partitions; blends span 11 union blocks), then
    shorter ones whose blends leave one, and two or three, whole union
    blocks in between."""
    spec = [(800_000, 1_300_000, 1), (50_000, 450_000, 2), (50_000, 450_000, 3),
            (120_000, 900_000, 4), (120_000, 900_000, 5)]
    parts = [gen.chain_around_walk(d, w, 64, 0x5EED00 + s, gen.BOX_INSET_ND) for d, w, s in spec]
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))


def deep_counts(kind, box):
    m, _, out, st = oracle.bbox(kind, box)
    assert st == 0
    far = cv.far_context_rows(kind, box, out, 8, 33)
    mid, levels = cv.mid_block_unions(kind, box, m, out)
    return dict(nonempty=int(cv.nonempty(out).sum()), far_ctx=far, mid_union=mid,
                mid_levels=sorted(levels))


def check_deep_counts(c, n):
    assert c["nonempty"] > 0.9 * n, c
    assert c["far_ctx"] >= 100_000, c
    assert c["mid_union"] >= 10_000, c
    assert set(c["mid_levels"]) >= {0, 1, 2, 3}, c


def c2_small():
    """The 2^27 headline scene's structure at 1/32 scale: a chain of 2^20
    opens around a 2^21-element walk, BOX_INSET boxes (5% of walk clips
    disjoint from their parent)."""
    return gen.chain_around_walk(1 << 20, 1 << 21, 64, 0x5EED14, gen.BOX_INSET)


def grad_scene():
    """A 400,000-element walk (cap 300, 391 partitions) on the 2^-8 grid with
    nested boxes: many ties, routes across partitions and through blends."""
    kind, box = gen.walk(400_000, 300, 0x5EED15, gen.BOX_INSET_ND)
    g = gen.normal(4 * len(kind), 0x5EED16).reshape(-1, 4)
    return kind, box, g


def grad_chain():
    """A chain of 40,000 opens (39 partitions) around a 40,000-element walk:
    gradients of deep rows route to clips dozens of partitions back."""
    kind, box = gen.chain_around_walk(40_000, 40_000, 30, 0x5EED17, gen.BOX_INSET_ND)
    g = gen.normal(4 * len(kind), 0x5EED18).reshape(-1, 4)
    return kind, box, g


# ------------------------------------------------------------ CPU: the inputs
def test_inputs_deep_scene_coverage():
    kind, box = deep_scene()
    c = deep_counts(kind, box)
    say(f"[coverage] deep scene n={len(kind)} {c}")
    check_deep_counts(c, len(kind))


def test_inputs_c2_small_coverage():
    kind, box = c2_small()
    m, _, out, st = oracle.bbox(kind, box)
    assert st == 0
    ne = cv.nonempty(out)
    assert ne.mean() > 0.5 and ne[kind == 0].mean() > 0.3
    assert cv.far_context_rows(kind, box, out, 8, 33) >= 100_000


def test_inputs_grad_coverage():
    kind, box, _ = grad_scene()
    far, blend, total = cv.cross_partition_routes(kind, box)
    far8, _, _ = cv.cross_partition_routes(kind, box, 8)
    say(f"[coverage] grad scene routes={total} cross-partition={far} via blends={blend} >=8 partitions={far8}")
    assert far >= 100_000 and blend >= 10_000 and far8 >= 10_000
    kind, box, _ = grad_chain()
    far33, _, total = cv.cross_partition_routes(kind, box, 33)
    assert far33 >= 1000, (far33, total)


# ------------------------------------------------------------ GPU parity
def check(kind, box, tag):
    say(f"[values] {tag} n={len(kind)}")
    m, out, st = gpu_bbox(kind, box)
    om, _, oout, ost = oracle.bbox(kind, box)
    assert ost == 0 and st == 0, (ost, st)
    bad = np.nonzero(m != om)[0]
    assert len(bad) == 0, f"{tag}: match differs at {bad[:10]}"
    badb = np.nonzero((out.view(np.uint32) != oout.view(np.uint32)).any(1))[0]
    assert len(badb) == 0, f"{tag}: box differs at {badb[:10]} kinds={kind[badb[:10]]}"


@pytest.mark.gpu
def test_deep_scene_values():
    kind, box = deep_scene()
    c = deep_counts(kind, box)
    say(f"[values] deep scene counts {c}")
    check_deep_counts(c, len(kind))
    check(kind, box, "deep scene")


@pytest.mark.gpu
def test_c2_structure_values():
    kind, box = c2_small()
    check(kind, box, "2^20 chain around 2^21 walk, inset boxes")


@pytest.mark.gpu
def test_c1_and_c3_values():
    c = gen.config(1, nested_boxes=True)
    check(c["kind"], c["box"], "16M chains, inset boxes")
    c = gen.config(3, nested_boxes=True)
    say(f"[values] batched n={len(c['kind'])}")
    m, out, st = gpu_batched(c["kind"], c["box"], c["offsets"])
    assert (st == 0).all()
    off = c["offsets"]
    nonempty = 0
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        om, _, oout, ost = oracle.bbox(c["kind"][a:b], c["box"][a:b])
        assert ost == 0
        assert np.array_equal(m[a:b], om) and same_bits(out[a:b], oout), s
        nonempty += int(cv.nonempty(oout).sum())
    say(f"[values] batched non-EMPTY rows {nonempty} of {len(c['kind'])}")
    assert nonempty > 0.2 * len(c["kind"])


def gpu_backward(kind, box, g):
    import torch
    import paper_2205_11659_amd as tb
    gi, st = tb.tb_bbox_backward(to_dev(kind), to_dev(box), to_dev(g))
    torch.cuda.synchronize()
    return gi.cpu().numpy(), int(st.item())


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["walk", "chain"])
def test_backward_values(which):
    kind, box, g = grad_scene() if which == "walk" else grad_chain()
    far, blend, total = cv.cross_partition_routes(kind, box, 1 if which == "walk" else 33)
    say(f"[values] backward {which} n={len(kind)} routes={total} far={far} via blends={blend}")
    assert far >= 1000
    gi, st = gpu_backward(kind, box, g)
    ogi, ost = oracle.backward(kind, box, g)
    assert st == 0 and ost == 0
    bad = np.nonzero((gi.view(np.uint32) != ogi.view(np.uint32)).any(1))[0]
    assert len(bad) == 0, f"grad differs at rows {bad[:10]}"
    assert (ogi != 0).sum() > len(kind) // 4
