"""Helpers for GPU tests: numpy <-> device and the library calls."""
import sys

import numpy as np


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_bbox(kind, box):
    import torch
    import paper_2205_11659_amd as tb
    out, m, st = tb.tb_bbox(to_dev(kind), to_dev(box))
    torch.cuda.synchronize()
    return m.cpu().numpy(), out.cpu().numpy(), int(st.item())


def gpu_match(kind):
    import torch
    import paper_2205_11659_amd as tb
    m, pm, st = tb.tb_match(to_dev(kind))
    torch.cuda.synchronize()
    return m.cpu().numpy(), pm.cpu().numpy(), int(st.item())


def gpu_batched(kind, box, offsets):
    import torch
    import paper_2205_11659_amd as tb
    out, m, st = tb.tb_bbox_batched(to_dev(kind), to_dev(box), to_dev(offsets))
    torch.cuda.synchronize()
    return m.cpu().numpy(), out.cpu().numpy(), st.cpu().numpy().view(np.uint32)


def same_bits(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint32), np.ascontiguousarray(b).view(np.uint32))
