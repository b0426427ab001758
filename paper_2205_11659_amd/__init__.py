"""libtreebbox: bounding boxes on flattened scene trees (arXiv 2205.11659)
for AMD Instinct MI355X.

Thin binding over the C ABI in include/treebbox.h: arguments are marshalled
from torch tensors (device memory, current HIP stream); every step of the
computation runs in the library's HIP kernels.  Importing works without a
GPU; calling requires the built library and a GPU.

    box_out, match, status = tb_bbox(kind, box)
    match, pm, status = tb_match(kind)
    box_out, match, status = tb_bbox_batched(kind, box, offsets)
    grad_in, status = tb_bbox_backward(kind, box, grad_out)
    box_out = bbox(kind, box)            # autograd-aware (TreeBBoxFn)
"""
import ctypes
import os

import torch

from ._build import LIB, build  # noqa: F401

LEAF, BEGIN_CLIP, END_CLIP, BEGIN_BLEND, END_BLEND, OTHER = range(6)
DATA_BAD_KIND, DATA_UNBALANCED, DATA_KIND_MISMATCH, DATA_BAD_OFFSETS, DATA_GRAD_RANGE = 1, 2, 4, 8, 16
_DATA_NAMES = {DATA_BAD_KIND: "BAD_KIND", DATA_UNBALANCED: "UNBALANCED",
               DATA_KIND_MISMATCH: "KIND_MISMATCH", DATA_BAD_OFFSETS: "BAD_OFFSETS",
               DATA_GRAD_RANGE: "GRAD_RANGE"}
(OP_MATCH, OP_BBOX, OP_BBOX_BACKWARD, OP_BBOX_BATCHED, OP_COMPOSE, OP_BBOX_STREAM, OP_COMPOSE_F32,
 OP_REDUCE_UP_F32) = range(8)

_lib = None


class TreeBBoxError(RuntimeError):
    pass


def lib():
    """The loaded libtreebbox.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise TreeBBoxError(f"libtreebbox.so not built ({LIB}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB)
        P, I64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
        L.tb_workspace_bytes.argtypes = [ctypes.c_int, I64, I64]
        L.tb_workspace_bytes.restype = SZ
        L.tb_match.argtypes = [P, I64, P, P, P, SZ, P, P]
        L.tb_bbox.argtypes = [P, P, I64, P, P, P, SZ, P, P]
        L.tb_match_brackets.argtypes = [P, I64, P, P, P, SZ, P, P]
        L.tb_compose_f32.argtypes = [P, P, I64, P, P, SZ, P, P]
        L.tb_compose_f32.restype = ctypes.c_int
        L.tb_reduce_up_f32.argtypes = [P, P, I64, P, P, SZ, P, P]
        L.tb_reduce_up_f32.restype = ctypes.c_int
        L.tb_match_brackets.restype = ctypes.c_int
        L.tb_bbox_backward.argtypes = [P, P, P, I64, P, P, SZ, P, P]
        L.tb_bbox_batched.argtypes = [P, P, P, I64, I64, P, P, P, SZ, P, P]
        L.tb_compose.argtypes = [P, P, I64, P, P, SZ, P, P]
        L.tb_bbox_stream.argtypes = [P, P, I64, P, P, P, SZ, P, P]
        L.tb_bbox_noalloc.argtypes = [P, P, I64, P, P, P, P]
        for f in (L.tb_match, L.tb_bbox, L.tb_bbox_backward, L.tb_bbox_batched, L.tb_compose,
                  L.tb_bbox_stream, L.tb_bbox_noalloc):
            f.restype = ctypes.c_int
        I32 = ctypes.c_int
        L.tb_tune_match.argtypes = [P, I64, P, P, P, SZ, P, P, I32, P, P]
        L.tb_tune_bbox.argtypes = [P, P, I64, P, P, P, SZ, P, P, I32, P, P]
        L.tb_tune_bbox_batched.argtypes = [P, P, P, I64, I64, P, P, P, SZ, P, P, I32, P, P]
        L.tb_variant_get.argtypes = [I32, I64, P]
        L.tb_variant_set.argtypes = [I32, I64, P]
        L.tb_tune_save.argtypes = [ctypes.c_char_p]
        L.tb_tune_load.argtypes = [ctypes.c_char_p]
        for f in (L.tb_tune_match, L.tb_tune_bbox, L.tb_tune_bbox_batched, L.tb_variant_get,
                  L.tb_variant_set, L.tb_tune_save, L.tb_tune_load):
            f.restype = I32
        L.tb_tune_clear.argtypes = []
        L.tb_tune_clear.restype = None
        L.tb_status_str.argtypes = [ctypes.c_int]
        L.tb_status_str.restype = ctypes.c_char_p
        _lib = L
    return _lib


# Workspaces are cached per (device, stream): calls on one stream are ordered,
# so they may share one; calls on different streams get different buffers.
# A buffer used while a HIP graph is being captured is written by every
# replay of that graph, so it is never freed or handed to another stream:
# it moves to _ws_pinned when the cache replaces it.
_ws_cache = {}
_ws_pinned = []


def workspace(op, n, num_scenes=1, device=None):
    """A device workspace of at least tb_workspace_bytes(op, n, S) bytes for
    the current stream (cached per device and stream; grown on demand)."""
    need = lib().tb_workspace_bytes(op, n, num_scenes)
    if need == 0:
        raise TreeBBoxError(f"invalid size for op {op}: n={n}, scenes={num_scenes}")
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    key = (dev, torch.cuda.current_stream(dev).cuda_stream)
    capturing = torch.cuda.is_current_stream_capturing()
    ent = _ws_cache.get(key)
    if ent is None or ent[0].numel() < need:
        if ent is not None and ent[1]:
            _ws_pinned.append(ent[0])
        ent = [torch.empty(need + 256, dtype=torch.uint8, device=dev), False]
        _ws_cache[key] = ent
    ent[1] = ent[1] or capturing
    buf = ent[0]
    ptr = buf.data_ptr()
    pad = (-ptr) % 256
    return ptr + pad, buf.numel() - pad


def status_bits(word):
    """Names of the TB_DATA_* bits set in a status word."""
    return [name for bit, name in _DATA_NAMES.items() if int(word) & bit]


def check_status(status, what="tb call"):
    """Raise TreeBBoxError if any status word is non-zero (synchronises)."""
    words = status.cpu().view(torch.int32).tolist()
    bad = [(i, w) for i, w in enumerate(words) if w != 0]
    if bad:
        i, w = bad[0]
        raise TreeBBoxError(f"{what}: data error {'|'.join(status_bits(w))} (status word {i} = {w:#x}"
                            f"; {len(bad)} word(s) non-zero)")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check(rc):
    if rc != 0:
        raise TreeBBoxError(lib().tb_status_str(rc).decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _as_kind(kind):
    if kind.dtype not in (torch.int32, torch.uint32):
        raise TypeError("kind must be int32/uint32")
    return kind.contiguous()


def _as_box(box, n):
    if box.dtype != torch.float32 or box.shape != (n, 4):
        raise TypeError("box must be float32 of shape (n, 4)")
    return box.contiguous()


def tb_match(kind, pm=True, match=None, status=None):
    """Matching only: returns (match int32[n], pm int32[n] or None, status int32[1]).
    `pm` may be True/False or a preallocated int32 tensor; `match` and
    `status` may be preallocated too."""
    kind = _as_kind(kind)
    n = kind.numel()
    dev = kind.device
    match = torch.empty(n, dtype=torch.int32, device=dev) if match is None else match
    if isinstance(pm, torch.Tensor):
        pmo = pm
    else:
        pmo = torch.empty(n, dtype=torch.int32, device=dev) if pm else None
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_MATCH, n, 1, dev)
    _check(lib().tb_match(_ptr(kind), n, _ptr(match), _ptr(pmo), ctypes.c_void_p(ws), wsb,
                          _ptr(status), _stream()))
    return match, pmo, status


def tb_match_brackets(tok, pm=True, match=None, status=None):
    """Typed bracket matching (token 0 none, 2t+1 open type t, 2t+2 close
    type t): returns (match int32[n], pm int32[n] or None, status int32[1])."""
    tok = _as_kind(tok)
    n = tok.numel()
    dev = tok.device
    match = torch.empty(n, dtype=torch.int32, device=dev) if match is None else match
    if isinstance(pm, torch.Tensor):
        pmo = pm
    else:
        pmo = torch.empty(n, dtype=torch.int32, device=dev) if pm else None
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_MATCH, n, 1, dev)
    _check(lib().tb_match_brackets(_ptr(tok), n, _ptr(match), _ptr(pmo), ctypes.c_void_p(ws), wsb,
                                   _ptr(status), _stream()))
    return match, pmo, status


def tb_bbox(kind, box, match=True, out=None, status=None):
    """Forward: returns (box_out float32[n,4], match int32[n] or None, status int32[1]).
    `match` may be True/False or a preallocated int32 tensor; `out` and
    `status` may be preallocated too."""
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    dev = kind.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev) if out is None else out
    if isinstance(match, torch.Tensor):
        m = match
    else:
        m = torch.empty(n, dtype=torch.int32, device=dev) if match else None
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_BBOX, n, 1, dev)
    _check(lib().tb_bbox(_ptr(kind), _ptr(box), n, _ptr(m), _ptr(out), ctypes.c_void_p(ws), wsb,
                         _ptr(status), _stream()))
    return out, m, status


NOALLOC_MAX_N = 1 << 20


def tb_bbox_noalloc(kind, box, match, out, status):
    """tb_bbox through the library's fixed per-GPU array instead of a
    workspace: the library allocates nothing, and neither does this wrapper
    (match, out and status are the caller's preallocated tensors; match may
    be None).  n <= NOALLOC_MAX_N.  Calls overlapping on one GPU race."""
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    _check(lib().tb_bbox_noalloc(_ptr(kind), _ptr(box), n, _ptr(match), _ptr(out), _ptr(status),
                                 _stream()))
    return out, match, status


def tb_bbox_batched(kind, box, offsets, match=True):
    """Ragged batch: offsets int64[S+1] on the device.  Returns
    (box_out, match (scene-local) or None, status int32[S])."""
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    offsets = offsets.contiguous()
    S = offsets.numel() - 1
    dev = kind.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    m = torch.empty(n, dtype=torch.int32, device=dev) if match else None
    status = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    ws, wsb = workspace(OP_BBOX_BATCHED, n, S, dev)
    _check(lib().tb_bbox_batched(_ptr(kind), _ptr(box), _ptr(offsets), S, n, _ptr(m), _ptr(out),
                                 ctypes.c_void_p(ws), wsb, _ptr(status), _stream()))
    return out, m, status


def tb_bbox_batched_into(kind, box, offsets, match, out, status):
    """tb_bbox_batched into the caller's preallocated match (or None), out
    and status (S words) tensors: nothing is allocated here except a larger
    cached workspace on first use, so it can be captured in a HIP graph."""
    kind = _as_kind(kind)
    n = kind.numel()
    S = offsets.numel() - 1
    ws, wsb = workspace(OP_BBOX_BATCHED, n, S, kind.device)
    _check(lib().tb_bbox_batched(_ptr(kind), _ptr(box), _ptr(offsets), S, n, _ptr(match), _ptr(out),
                                 ctypes.c_void_p(ws), wsb, _ptr(status), _stream()))
    return out, match, status


def tb_bbox_backward(kind, box, grad_out):
    """Gradient of tb_bbox's box output w.r.t. box: returns (grad_in, status)."""
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    grad_out = _as_box(grad_out, n)
    dev = kind.device
    gin = torch.empty((n, 4), dtype=torch.float32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    ws, wsb = workspace(OP_BBOX_BACKWARD, n, 1, dev)
    _check(lib().tb_bbox_backward(_ptr(kind), _ptr(box), _ptr(grad_out), n, _ptr(gin),
                                  ctypes.c_void_p(ws), wsb, _ptr(status), _stream()))
    return gin, status


def tb_compose(kind, xf, out=None, status=None):
    """Transforms composed down the tree.  `xf` holds int32[n, 6] rows
    [a b c d e f] read as uint32 modulo 2^32 (rows of opens are used).
    Returns (out int32[n, 6], status int32[1])."""
    kind = _as_kind(kind)
    n = kind.numel()
    if xf.dtype != torch.int32 or xf.shape != (n, 6):
        raise TypeError("xf must be int32 [n, 6]")
    xf = xf.contiguous()
    dev = kind.device
    out = torch.empty((n, 6), dtype=torch.int32, device=dev) if out is None else out
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_COMPOSE, n, 1, dev)
    _check(lib().tb_compose(_ptr(kind), _ptr(xf), n, _ptr(out), ctypes.c_void_p(ws), wsb,
                            _ptr(status), _stream()))
    return out, status


def tb_compose_f32(kind, xf, out=None, status=None):
    """fp32 transforms composed down the tree in pointer-jumping order.
    `xf` float32[n, 6] rows [a b c d e f] (rows of opens used).  Returns
    (out float32[n, 6], status int32[1])."""
    kind = _as_kind(kind)
    n = kind.numel()
    if xf.dtype != torch.float32 or xf.shape != (n, 6):
        raise TypeError("xf must be float32 [n, 6]")
    xf = xf.contiguous()
    dev = kind.device
    out = torch.empty((n, 6), dtype=torch.float32, device=dev) if out is None else out
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_COMPOSE_F32, n, 1, dev)
    _check(lib().tb_compose_f32(_ptr(kind), _ptr(xf), n, _ptr(out), ctypes.c_void_p(ws), wsb,
                                _ptr(status), _stream()))
    return out, status


def tb_reduce_up_f32(kind, xf, out=None, status=None):
    """fp32 transforms of the leaves multiplied up the tree in sequence order
    (segment-tree grouping).  `xf` float32[n, 6] (rows of leaves used).
    Returns (out float32[n, 6], status int32[1])."""
    kind = _as_kind(kind)
    n = kind.numel()
    if xf.dtype != torch.float32 or xf.shape != (n, 6):
        raise TypeError("xf must be float32 [n, 6]")
    xf = xf.contiguous()
    dev = kind.device
    out = torch.empty((n, 6), dtype=torch.float32, device=dev) if out is None else out
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_REDUCE_UP_F32, n, 1, dev)
    _check(lib().tb_reduce_up_f32(_ptr(kind), _ptr(xf), n, _ptr(out), ctypes.c_void_p(ws), wsb,
                                  _ptr(status), _stream()))
    return out, status


def tb_bbox_stream(tag, box, match=True, out=None, status=None):
    """Node boxes over a draw-object stream: tags 0..4 are the tree's
    elements, OTHER (5) marks elements outside the tree.  Returns (box_out
    float32[n,4], match int32[n] or None, status int32[1]); rows and match
    entries at OTHER positions are not written, so pass preallocated `out`
    and `match` tensors to keep values there."""
    tag = _as_kind(tag)
    n = tag.numel()
    box = _as_box(box, n)
    dev = tag.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev) if out is None else out
    if isinstance(match, torch.Tensor):
        m = match
    else:
        m = torch.empty(n, dtype=torch.int32, device=dev) if match else None
    status = torch.empty(1, dtype=torch.int32, device=dev) if status is None else status
    ws, wsb = workspace(OP_BBOX_STREAM, n, 1, dev)
    _check(lib().tb_bbox_stream(_ptr(tag), _ptr(box), n, _ptr(m), _ptr(out), ctypes.c_void_p(ws),
                                wsb, _ptr(status), _stream()))
    return out, m, status


# ---------------------------------------------------------------- tuning
class Variant(ctypes.Structure):
    """Launch variant: elements per thread of the main and the reduce pass,
    close records per thread of the cross-partition pass."""
    _fields_ = [("resolve_elems", ctypes.c_int32), ("reduce_elems", ctypes.c_int32),
                ("cross_records", ctypes.c_int32)]

    def astuple(self):
        return (self.resolve_elems, self.reduce_elems, self.cross_records)


def variant_get(op, n):
    v = Variant()
    _check(lib().tb_variant_get(op, n, ctypes.byref(v)))
    return v.astuple()


def variant_set(op, n, v):
    """Pin the variant (a 3-tuple) for n's size class; None restores the default."""
    if v is None:
        _check(lib().tb_variant_set(op, n, None))
    else:
        _check(lib().tb_variant_set(op, n, ctypes.byref(Variant(*v))))


def tune_save(path):
    _check(lib().tb_tune_save(os.fsencode(path)))


def tune_load(path):
    _check(lib().tb_tune_load(os.fsencode(path)))


def tune_clear():
    lib().tb_tune_clear()


def _tuned(rc, v, ms):
    _check(rc)
    return {"variant": v.astuple(), "ms": float(ms[0]), "default_ms": float(ms[1])}


def tune_bbox(kind, box, reps=3):
    """Time every tb_bbox variant on this input, keep the fastest for its
    size class; returns {variant, ms, default_ms} and the call's outputs."""
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    dev = kind.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    m = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    ws, wsb = workspace(OP_BBOX, n, 1, dev)
    v, ms = Variant(), (ctypes.c_float * 2)()
    rc = lib().tb_tune_bbox(_ptr(kind), _ptr(box), n, _ptr(m), _ptr(out), ctypes.c_void_p(ws), wsb,
                            _ptr(status), _stream(), reps, ctypes.byref(v), ms)
    return _tuned(rc, v, ms), (out, m, status)


def tune_bbox_batched(kind, box, offsets, reps=3):
    kind = _as_kind(kind)
    n = kind.numel()
    box = _as_box(box, n)
    offsets = offsets.contiguous()
    S = offsets.numel() - 1
    dev = kind.device
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    m = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    ws, wsb = workspace(OP_BBOX_BATCHED, n, S, dev)
    v, ms = Variant(), (ctypes.c_float * 2)()
    rc = lib().tb_tune_bbox_batched(_ptr(kind), _ptr(box), _ptr(offsets), S, n, _ptr(m), _ptr(out),
                                    ctypes.c_void_p(ws), wsb, _ptr(status), _stream(), reps,
                                    ctypes.byref(v), ms)
    return _tuned(rc, v, ms), (out, m, status)


def tune_match(kind, reps=3):
    kind = _as_kind(kind)
    n = kind.numel()
    dev = kind.device
    m = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    ws, wsb = workspace(OP_MATCH, n, 1, dev)
    v, ms = Variant(), (ctypes.c_float * 2)()
    rc = lib().tb_tune_match(_ptr(kind), n, _ptr(m), None, ctypes.c_void_p(ws), wsb, _ptr(status),
                             _stream(), reps, ctypes.byref(v), ms)
    return _tuned(rc, v, ms), (m, status)


def candidates(op):
    """Every launch variant the tuner tries for `op`."""
    boxes = op != OP_MATCH
    return [(kr, kd, cu) for kr in (4, 8) for kd in (4, 8) for cu in (2, 4, 8) if boxes or cu == 4]


class TreeBBoxFn(torch.autograd.Function):
    """(box_out, match, status) = TreeBBoxFn.apply(kind, box, check).

    match and status are non-differentiable.  With check=True the forward
    raises TreeBBoxError on a non-zero status word (malformed scene), and the
    backward raises on a non-zero status of its own pass (e.g. an upstream
    gradient out of range); each check synchronises the stream.  With
    check=False the status words are only returned, and reading them is the
    caller's job."""

    @staticmethod
    def forward(ctx, kind, box, check=True):
        out, match, status = tb_bbox(kind, box)
        if check:
            check_status(status, "tb_bbox")
        ctx.save_for_backward(kind, box)
        ctx.check = check
        ctx.mark_non_differentiable(match, status)
        return out, match, status

    @staticmethod
    def backward(ctx, g_out, _g_match, _g_status):
        kind, box = ctx.saved_tensors
        gin, status = tb_bbox_backward(kind, box, g_out.contiguous())
        if ctx.check:
            check_status(status, "tb_bbox_backward")
        return None, gin, None


def bbox(kind, box, check=True):
    """Node boxes through TreeBBoxFn (autograd-aware); raises on malformed
    input unless check=False."""
    out, _, _ = TreeBBoxFn.apply(kind, box, check)
    return out


class PerSceneGraph:
    """One tb_bbox call per scene, captured once into a HIP graph (the
    baseline that tb_bbox_batched is compared with).  Outputs are views of
    one (n, 4) box buffer and one int32 match buffer, so the rows line up
    with the batched call's; status holds one word per scene."""

    def __init__(self, kind, box, offsets_host):
        n = kind.numel()
        dev = kind.device
        self.kind, self.box = _as_kind(kind), _as_box(box, n)
        self.out = torch.empty((n, 4), dtype=torch.float32, device=dev)
        self.match = torch.empty(n, dtype=torch.int32, device=dev)
        S = len(offsets_host) - 1
        self.status = torch.zeros(max(S, 1), dtype=torch.int32, device=dev)
        offs = [int(v) for v in offsets_host]
        big = max([b - a for a, b in zip(offs[:-1], offs[1:])] + [0])
        need = lib().tb_workspace_bytes(OP_BBOX, big, 1)
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        wsp = self.ws.data_ptr() + ((-self.ws.data_ptr()) % 256)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(self.graph, stream=side):
                st = _stream()
                for s in range(S):
                    a, b = offs[s], offs[s + 1]
                    _check(lib().tb_bbox(
                        ctypes.c_void_p(self.kind.data_ptr() + 4 * a),
                        ctypes.c_void_p(self.box.data_ptr() + 16 * a), b - a,
                        ctypes.c_void_p(self.match.data_ptr() + 4 * a),
                        ctypes.c_void_p(self.out.data_ptr() + 16 * a),
                        ctypes.c_void_p(wsp), need,
                        ctypes.c_void_p(self.status.data_ptr() + 4 * s), st))
        torch.cuda.current_stream().wait_stream(side)

    def replay(self):
        self.graph.replay()
        return self.out, self.match, self.status
