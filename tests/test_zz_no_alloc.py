"""tb_bbox_noalloc (no workspace, nothing allocated) against tb_bbox, bit
for bit, on two calls in a row through the C ABI, the second smaller; and
the size limit."""
import ctypes

import numpy as np
import pytest

import gen
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu


def _run_both(tb, kind_np, box_np):
    import torch
    n = len(kind_np)
    kind, box = to_dev(kind_np), to_dev(box_np)
    dev = kind.device
    out = torch.full((n, 4), float("nan"), dtype=torch.float32, device=dev)
    m = torch.full((n,), -7, dtype=torch.int32, device=dev)
    st = torch.full((1,), -1, dtype=torch.int32, device=dev)
    tb.tb_bbox_noalloc(kind, box, m, out, st)
    ref_out, ref_m, ref_st = tb.tb_bbox(kind, box)
    torch.cuda.synchronize()
    return (out.cpu().numpy(), m.cpu().numpy(), int(st.item()),
            ref_out.cpu().numpy(), ref_m.cpu().numpy(), int(ref_st.item()))


def test_noalloc_matches_tb_bbox_twice():
    import paper_2205_11659_amd as tb
    # a full-size call (the maximum), then a smaller, ragged one
    for n, seed in ((tb.NOALLOC_MAX_N, 0x0A11), (70_001, 0x0A12)):
        kind, box = gen.walk(n, 64, seed, gen.BOX_INSET)
        say(f"[noalloc] n={n}")
        out, m, st, rout, rm, rst = _run_both(tb, kind, box)
        assert st == 0 and rst == 0
        assert np.array_equal(m, rm)
        assert np.array_equal(out.view(np.uint32), rout.view(np.uint32))


def test_noalloc_null_match_and_deep_chain():
    import torch
    import paper_2205_11659_amd as tb
    kind_np, box_np = gen.chain_around_walk(200_000, 300_000, 64, 0x0A13, gen.BOX_INSET_ND)
    n = len(kind_np)
    say(f"[noalloc] chain n={n}, match NULL")
    kind, box = to_dev(kind_np), to_dev(box_np)
    out = torch.empty((n, 4), dtype=torch.float32, device=kind.device)
    st = torch.empty(1, dtype=torch.int32, device=kind.device)
    tb.tb_bbox_noalloc(kind, box, None, out, st)
    ref_out, _, ref_st = tb.tb_bbox(kind, box, match=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and int(ref_st.item()) == 0
    assert torch.equal(out.view(torch.int32), ref_out.view(torch.int32))


def test_noalloc_rejects_too_large():
    import paper_2205_11659_amd as tb
    L = tb.lib()
    rc = L.tb_bbox_noalloc(ctypes.c_void_p(16), ctypes.c_void_p(16), tb.NOALLOC_MAX_N + 1,
                           ctypes.c_void_p(0), ctypes.c_void_p(16), ctypes.c_void_p(16),
                           ctypes.c_void_p(0))
    assert rc == 7
    assert b"2^20" in L.tb_status_str(7)
