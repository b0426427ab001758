"""GPU status words: data errors are reported per scene exactly as the
oracle reports them, the autograd path raises on them, and the gradient
pass flags upstream gradients it cannot represent."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import gpu_batched, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("trailing_empty", [0, 2])
def test_unbalanced_last_scene(trailing_empty):
    """The last non-empty scene ends with an open never closed, and the total
    length is not a multiple of the partition size: only that scene's word
    reports UNBALANCED, as the oracle does for it alone."""
    kind, box, off = gen.batch(25, 5.0, 11.0, 2, 60, 0x57A7, gen.BOX_INSET)
    last = len(off) - 2
    a = off[last]
    kind = np.concatenate([kind[:a], [1], kind[a:]]).astype(np.uint32)  # extra open at its start
    box = np.concatenate([box[:a], [[0, 0, 1, 1]], box[a:]]).astype(np.float32)
    off = off.copy()
    off[-1] += 1
    off = np.concatenate([off, [off[-1]] * trailing_empty]).astype(np.int64)
    n = len(kind)
    assert n % 1024 != 0
    say(f"[status] unbalanced last scene n={n} scenes={len(off) - 1}")
    m, out, st = gpu_batched(kind, box, off)
    for s in range(len(off) - 1):
        x, y = off[s], off[s + 1]
        _, _, _, ost = oracle.bbox(kind[x:y], box[x:y])
        assert st[s] == ost, (s, st[s], ost)
    assert st[last] & 2


def test_bad_offsets_flag_every_scene():
    kind, box, off = gen.batch(12, 4.0, 9.0, 2, 30, 0x57A8)
    n = len(kind)
    cases = []
    o1 = off.copy(); o1[3], o1[4] = o1[4], o1[3]  # not monotone
    cases.append(o1)
    o2 = off.copy(); o2[-1] = n - 1  # does not end at n
    cases.append(o2)
    o3 = off.copy(); o3[0] = 1  # does not start at 0
    cases.append(o3)
    for o in cases:
        say(f"[status] bad offsets {o[:6]}...")
        _, _, st = gpu_batched(kind, box, o.astype(np.int64))
        assert (st & 8).all(), st


def test_autograd_raises_on_malformed_scene():
    import torch
    import paper_2205_11659_amd as tb
    kind, box = gen.walk(3000, 20, 0x57A9, gen.BOX_INSET)
    kind = np.concatenate([[1], kind]).astype(np.uint32)  # an open never closed
    box = np.concatenate([[[0, 0, 1, 1]], box]).astype(np.float32)
    say("[status] autograd on a malformed scene")
    bt = to_dev(box).requires_grad_(True)
    with pytest.raises(tb.TreeBBoxError, match="UNBALANCED"):
        tb.bbox(to_dev(kind), bt)
    out = tb.bbox(to_dev(kind), bt, check=False)  # unchecked: returns, status left to the caller
    torch.cuda.synchronize()
    assert out.shape == (len(kind), 4)


def test_backward_grad_range():
    import torch
    import paper_2205_11659_amd as tb
    kind, box = gen.walk(5000, 30, 0x57AA, gen.BOX_INSET_ND)
    n = len(kind)
    g = gen.normal(4 * n, 0x57AB).reshape(n, 4)
    leaf = int(np.flatnonzero(kind == 0)[10])
    g[leaf, 0] = np.float32(3e9)  # routed (every leaf is non-empty): out of range
    say("[status] backward with |g| >= 2^31")
    gi, st = tb.tb_bbox_backward(to_dev(kind), to_dev(box), to_dev(g))
    torch.cuda.synchronize()
    _, ost = oracle.backward(kind, box, g)
    assert ost == 16 and int(st.item()) == 16
    bt = to_dev(box).requires_grad_(True)
    out = tb.bbox(to_dev(kind), bt)
    with pytest.raises(tb.TreeBBoxError, match="GRAD_RANGE"):
        out.backward(to_dev(g))
