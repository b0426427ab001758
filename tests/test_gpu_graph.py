"""Per-scene calls captured in one HIP graph give byte-identical rows to one
tb_bbox_batched call; every replay is checked, with eager work between."""
import numpy as np
import pytest

import gen
from gpu_util import dev, same_bits, say, to_dev

pytestmark = pytest.mark.gpu


def test_graph_per_scene_equals_batched():
    import torch
    import paper_2205_11659_amd as tb
    kind, box, off = gen.batch(300, 4.0, 13.0, 2, 800, 6100, gen.BOX_NESTED_ALL)
    say(f"[graph] scenes=300 n={len(kind)}")
    k, b, o = to_dev(kind), to_dev(box), to_dev(off)
    bout, bm, bst = tb.tb_bbox_batched(k, b, o)
    torch.cuda.synchronize()
    assert (bst.cpu().numpy() == 0).all()
    g = tb.PerSceneGraph(k, b, off)
    ref_out, ref_m = bout.cpu().numpy(), bm.cpu().numpy()
    for rep in range(3):
        out, m, st = g.replay()
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == 0).all()
        assert same_bits(out.cpu().numpy(), ref_out), f"replay {rep}: boxes differ"
        assert np.array_equal(m.cpu().numpy(), ref_m), f"replay {rep}: match differs"
        # eager work between replays, on the same buffers' device
        junk = torch.randn(1 << 20, device=dev()).sum()
        torch.cuda.synchronize()
        del junk


def test_graph_stream_replays():
    """tb_bbox_stream enqueues no host synchronisation: captured once in a
    HIP graph, every replay recomputes the stream (outputs are reset
    eagerly between replays) and matches the oracle bit for bit."""
    import torch
    import oracle
    import paper_2205_11659_amd as tb
    k, b = gen.walk(60_000, 64, 6200, gen.BOX_NESTED_ALL)
    tag, sbox, _ = gen.interleave(k, b, 250_001, 6201)
    n = tag.shape[0]
    say(f"[graph] stream n={n} tree={len(k)}")
    t_d, b_d = to_dev(tag), to_dev(sbox)
    out = torch.full((n, 4), float("nan"), dtype=torch.float32, device=dev())
    m = torch.full((n,), -7, dtype=torch.int32, device=dev())
    st = torch.zeros(1, dtype=torch.int32, device=dev())
    tb.tb_bbox_stream(t_d, b_d, match=m, out=out, status=st)  # sizes the workspace
    torch.cuda.synchronize()
    om, oout, ost = oracle.bbox_stream(tag, sbox)
    assert ost == 0 and int(st.item()) == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            tb.tb_bbox_stream(t_d, b_d, match=m, out=out, status=st)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(float("nan"))
        m.fill_(-7)
        st.fill_(5)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0, f"replay {rep}: status"
        assert np.array_equal(m.cpu().numpy(), om), f"replay {rep}: match differs"
        assert same_bits(out.cpu().numpy(), oout), f"replay {rep}: boxes differ"
        junk = torch.randn(1 << 20, device=dev()).sum()
        torch.cuda.synchronize()
        del junk
