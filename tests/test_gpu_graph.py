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
