"""Benchmark: match + bbox forward on the 2^27-element deep-chain scene.

python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one tb_bbox call (matching, clip intersections, blend unions:
every kernel of the forward path) over the whole scene, inputs resident in
HBM.  Prints one JSON line.  The dominant kernel's duration is read live
with HIP events recorded on the call's stream around its launch.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALG_BYTES_FWD = 40  # kind 4 + box 16 in; match 4 + box 16 out
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_resolve_scene128M_traffic.json")


def kernel_source_hash():
    """Hash of the HIP sources the measured kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2205_11659_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel
    calibration), or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return int(round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024))


class HipEvents:
    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
        return e

    def elapsed_ms(self, a, b):
        self.hip.hipEventSynchronize(b)
        ms = ctypes.c_float()
        assert self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b) == 0
        return ms.value


def cpu_baseline(kind_np, box_np, budget_s=15.0):
    """The oracle (single-threaded sequential walk) on the same scene the GPU
    leg times, repeated until about budget_s of CPU time has been spent."""
    import oracle
    n = len(kind_np)
    times = []
    t_all = time.perf_counter()
    while len(times) < 2 or time.perf_counter() - t_all < budget_s:
        t0 = time.perf_counter()
        oracle.bbox(kind_np, box_np)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    return {"value": round(n / med / 1e9, 4), "unit": "Gelem/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole timed scene ({n} elements), median of {len(times)} runs, "
                      f"{med:.3f} s each, {sum(times):.1f} s in all"}


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def oracle_scenes_threads(kind_np, box_np, offsets, reps=3):
    """The oracle over the scenes of a batch on a thread pool (ctypes releases
    the GIL during each call), one scene per task; median of `reps` passes."""
    import concurrent.futures

    import oracle
    try:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        threads = max(1, min(16, os.cpu_count() or 1))
    S = len(offsets) - 1

    def one(sc):
        a, b = int(offsets[sc]), int(offsets[sc + 1])
        oracle.bbox(kind_np[a:b], box_np[a:b])

    order = np.argsort(-np.diff(np.asarray(offsets)), kind="stable")  # largest scenes first
    times = []
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(one, order.tolist()))
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    n = int(offsets[-1])
    return {"value": round(n / med / 1e9, 4), "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "sample": f"all {S} scenes ({n} elements), one scene per task, largest first, "
                      f"median of {reps} passes"}


def small_section(reps=100):
    """The 65,536-element scene (cap 64): launch-latency bound, so one tb_bbox
    call is captured in a HIP graph and replayed `reps` times."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(0)
    n = len(c["kind"])
    kind, box = torch.from_numpy(c["kind"].view(np.int32)).cuda(), torch.from_numpy(c["box"]).cuda()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    match = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    tuned = tb.tune_bbox(kind, box, reps=5)[0] if TUNE else None  # untimed: picks the launch variant
    tb.tb_bbox(kind, box, match=match, out=out, status=st)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            tb.tb_bbox(kind, box, match=match, out=out, status=st)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(5):
        graph.replay()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    us = a.elapsed_time(b) * 1e3 / reps
    return {"workload": c["name"], "elements": n, "us_per_call": round(us, 2),
            "gelem_s": round(n / us / 1e3, 3), "timing": f"HIP graph of one call, {reps} replays",
            "autotune": _tune_record(tuned) if tuned else None}


def copy_ceiling(reps=10):
    """A plain device copy of 1 GiB (read + write) timed with HIP events: the
    practical bandwidth ceiling beside the 8 TB/s peak.  The same copy,
    profiled with the FETCH_SIZE and WRITE_SIZE counters (`--only copy`),
    calibrates those counters: true bytes / counted bytes per dispatch."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    nbytes = 2 * src.numel() * 4
    del src, dst
    return {"gbs": round(nbytes / (ms / 1e3) / 1e9, 1), "bytes_moved": nbytes,
            "bytes_read_per_copy": nbytes // 2, "frac_of_peak": round(nbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


TUNE = True  # sections run the autotuner before timing (off for counter runs)


def _tune_record(t):
    """The autotuner's choice for a section: variant (elements per thread of
    the main and the reduce pass, close records per thread of the cross
    pass) and its median time against the default variant's."""
    return {"variant": list(t["variant"]), "ms": round(t["ms"], 4),
            "default_ms": round(t["default_ms"], 4),
            "gain": round(t["default_ms"] / t["ms"], 4) if t["ms"] > 0 else None}


def gpu_clocks():
    """Current engine (sclk) and memory (mclk) clock levels of the AMD GPUs,
    read from the driver's sysfs tables (the level marked '*' is current);
    no subprocess, so it also works under a profiler."""
    import glob
    out = {}
    try:
        for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
            try:
                if open(os.path.join(dev, "vendor")).read().strip() != "0x1002":
                    continue
            except OSError:
                continue
            card = {}
            for clk in ("pp_dpm_sclk", "pp_dpm_mclk", "pp_dpm_fclk"):
                try:
                    lines = open(os.path.join(dev, clk)).read().splitlines()
                except OSError:
                    continue
                cur = [ln.split(":", 1)[1].replace("*", "").strip() for ln in lines if "*" in ln]
                card[clk[7:]] = cur[0] if cur else None
            if card:
                out[os.path.basename(os.path.dirname(dev))] = card
    except Exception as e:  # unexpected sysfs content is reported, not fatal
        return {"error": str(e)[:200]}
    return out or {"error": "no AMD GPU clock tables in sysfs"}


def c1_section(steps, warmup):
    """The 2^24-element scene with 16 chains of depth 100,000 in a cap-16
    walk: forward throughput (reported, not graded)."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(1)
    n = len(c["kind"])
    kind, box = torch.from_numpy(c["kind"].view(np.int32)).cuda(), torch.from_numpy(c["box"]).cuda()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    m = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_bbox(kind, box, match=m, out=out, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": c["name"], "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(ALG_BYTES_FWD * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def batched_section(steps, warmup, cpu=False):
    """2048 ragged scenes: one tb_bbox_batched launch vs one graph-captured
    tb_bbox call per scene (same rows, byte-compared)."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(3)
    n = len(c["kind"])
    kind, box = torch.from_numpy(c["kind"].view(np.int32)).cuda(), torch.from_numpy(c["box"]).cuda()
    off = torch.from_numpy(c["offsets"]).cuda()
    out = {}
    tuned = tb.tune_bbox_batched(kind, box, off, reps=3)[0] if TUNE else None
    ms_b = time_steps(lambda: tb.tb_bbox_batched(kind, box, off), steps, warmup)
    bout, bm, bst = tb.tb_bbox_batched(kind, box, off)
    # the same batched call captured once in a HIP graph and replayed (the
    # paper excludes launch overhead; so does this figure)
    bo2 = torch.empty_like(bout)
    bm2 = torch.empty_like(bm)
    bs2 = torch.empty_like(bst)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    bgraph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(bgraph, stream=side):
            tb.tb_bbox_batched_into(kind, box, off, bm2, bo2, bs2)
    torch.cuda.current_stream().wait_stream(side)
    ms_bg = time_steps(bgraph.replay, steps, warmup)
    g = tb.PerSceneGraph(kind, box, c["offsets"])
    ms_g = time_steps(g.replay, steps, warmup)
    gout, gm, gst = g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(bout.view(torch.int32), gout.view(torch.int32)) and torch.equal(bm, gm)
                and int(bst.abs().sum()) == 0 and int(gst.abs().sum()) == 0)
    out.update({"workload": "batch-2048-ragged", "elements": n, "scenes": len(c["offsets"]) - 1,
                "batched_ms": round(ms_b, 4), "batched_gelem_s": round(n / ms_b / 1e6, 3),
                "batched_graph_ms": round(ms_bg, 4), "batched_graph_gelem_s": round(n / ms_bg / 1e6, 3),
                "graph_identical": bool(torch.equal(bo2.view(torch.int32), bout.view(torch.int32))
                                        and torch.equal(bm2, bm)),
                "per_scene_graph_ms": round(ms_g, 4), "per_scene_graph_gelem_s": round(n / ms_g / 1e6, 3),
                "speedup": round(ms_g / ms_b, 3), "byte_identical": same,
                "autotune": _tune_record(tuned) if tuned else None})
    if cpu:
        out["cpu_baseline_threads"] = oracle_scenes_threads(c["kind"], c["box"], c["offsets"])
    return out


def fwd_bwd_section(steps, warmup):
    """Forward + backward on the 2^24-element gradient workload, through the
    autograd.Function (TreeBBoxFn): out = bbox(kind, box); out.backward(g).
    Status checks are off inside the timed loop (each would synchronise);
    the status words are checked once after it."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(4)
    n = len(c["kind"])
    kind = torch.from_numpy(c["kind"].view(np.int32)).cuda()
    box = torch.from_numpy(c["box"]).cuda().requires_grad_(True)
    g = torch.from_numpy(c["grad"]).cuda()

    def step():
        box.grad = None
        out, _, st = tb.TreeBBoxFn.apply(kind, box, False)
        out.backward(g)
        return st

    ms = time_steps(step, steps, warmup)
    st = step()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ms_f = time_steps(lambda: tb.TreeBBoxFn.apply(kind, box.detach(), False), steps, warmup)
    return {"workload": "scene-16M-cap256-grad", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(92 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "forward_only_ms": round(ms_f, 4), "via": "TreeBBoxFn (autograd)"}


def match_section(steps, warmup, kind_np=None):
    """tb_match alone (the paper's own accounting: 4 B kind in, 4 B match
    out per element) on the same 2^27-element scene."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    if kind_np is None:
        kind_np = gen.config(2)["kind"]
    n = len(kind_np)
    kind = torch.from_numpy(kind_np.view(np.int32)).cuda()
    m = torch.empty(n, dtype=torch.int32, device="cuda")
    pm = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    tuned = tb.tune_match(kind, reps=9)[0] if TUNE else None  # variants differ by a few percent
    ms = time_steps(lambda: tb.tb_match(kind, pm=False, match=m, status=st), steps, warmup)
    ms_pm = time_steps(lambda: tb.tb_match(kind, pm=pm, match=m, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": "scene-128M-chain32M", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(8 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "with_pm_ms": round(ms_pm, 4), "autotune": _tune_record(tuned) if tuned else None,
            "context": "the paper reports 13.5 Gelem/s for matching alone on a Radeon 5700 XT"}


def brackets_section(steps, warmup):
    """tb_match_brackets on 2^27 typed bracket tokens (8 types, depth cap 64,
    about half the tokens brackets): 4 B token in, 4 B match out."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    n = 1 << 27
    tok_np = gen.brackets(n, 64, 8, gen.SEED_BASE + 32)
    tok = torch.from_numpy(tok_np.view(np.int32)).cuda()
    del tok_np
    m = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_match_brackets(tok, pm=False, match=m, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": "brackets-128M-8types-cap64", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(8 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def compose_section(steps, warmup, kind_np=None):
    """tb_compose (transforms composed down the tree) on the same scene:
    kind 4 B + transform 24 B in, transform 24 B out per element."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    if kind_np is None:
        kind_np = gen.config(2)["kind"]
    n = len(kind_np)
    kind = torch.from_numpy(kind_np.view(np.int32)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(gen.SEED_BASE + 2)
    xf = torch.randint(-(1 << 31), (1 << 31) - 1, (n, 6), dtype=torch.int32, device="cuda", generator=g)
    out = torch.empty_like(xf)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_compose(kind, xf, out=out, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": "scene-128M-chain32M", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(52 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def compose_f32_section(steps, warmup):
    """tb_compose_f32 (fp32 transforms, pointer-jumping order) on a 2^24
    cap-256 walk: matching, then ceil(log2(depth + 1)) rounds over all
    elements; algorithmic bytes: kind 4 + transform 24 in, transform 24 out."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(4)
    n = len(c["kind"])
    kind = torch.from_numpy(c["kind"].view(np.int32)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(gen.SEED_BASE + 40)
    xf = torch.rand((n, 6), generator=g, device="cuda") * 2 - 1
    out = torch.empty_like(xf)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_compose_f32(kind, xf, out=out, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": "scene-16M-cap256", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(52 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def reduce_up_f32_section(steps, warmup):
    """tb_reduce_up_f32 (leaves' fp32 transforms multiplied up the tree,
    segment-tree grouping) on the 2^24 cap-256 walk; algorithmic bytes:
    kind 4 + transform 24 in, transform 24 out per element."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    c = gen.config(4)
    n = len(c["kind"])
    kind = torch.from_numpy(c["kind"].view(np.int32)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(gen.SEED_BASE + 41)
    xf = torch.rand((n, 6), generator=g, device="cuda") * 2 - 1
    out = torch.empty_like(xf)
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_reduce_up_f32(kind, xf, out=out, status=st), steps, warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return {"workload": "scene-16M-cap256", "elements": n, "ms_per_step": round(ms, 4),
            "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(52 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def stream_section(steps, warmup):
    """tb_bbox_stream on a draw-object stream of 2^27 elements holding a
    cap-64 random-walk tree of 2^24 elements (density 1/8).  Algorithmic
    bytes: every tag read once (4 B per stream element); per tree element its
    box read, its row written (16 B each) and its partner written (4 B).  The
    same tree already extracted, through tb_bbox, is timed beside it."""
    import torch

    import gen
    import paper_2205_11659_amd as tb
    w = gen.stream_config()
    tag_np, box_np, m = w["tag"], w["box"], w["m"]
    n = len(tag_np)
    tag = torch.from_numpy(tag_np.view(np.int32)).cuda()
    box = torch.from_numpy(box_np).cuda()
    out = torch.empty_like(box)
    match = torch.empty(n, dtype=torch.int32, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    ms = time_steps(lambda: tb.tb_bbox_stream(tag, box, match=match, out=out, status=st), steps,
                    warmup)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    sel = tag_np <= 4
    kind = torch.from_numpy(tag_np[sel].view(np.int32)).cuda()
    cbox = torch.from_numpy(box_np[sel]).cuda()
    del tag, box, out, match
    cout = torch.empty_like(cbox)
    cmatch = torch.empty(m, dtype=torch.int32, device="cuda")
    ms_c = time_steps(lambda: tb.tb_bbox(kind, cbox, match=cmatch, out=cout, status=st), steps,
                      warmup)
    torch.cuda.synchronize()
    alg = 4 * n + 36 * m
    return {"workload": w["name"], "elements": n, "tree_elements": m,
            "ms_per_step": round(ms, 4), "gelem_s": round(n / ms / 1e6, 3),
            "hbm_frac_alg": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "extracted_tree_alone_ms": round(ms_c, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="time the default launch variant")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and fwd+bwd sections")
    ap.add_argument("--only", choices=["stream", "match", "compose", "batched", "fwd_bwd", "small",
                                       "c1", "copy", "brackets", "compose_f32", "reduce_up_f32"],
                    help="run one secondary section alone and print its JSON (for profiling)")
    args = ap.parse_args()
    global TUNE
    TUNE = not args.no_tune
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the path has no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    if args.only:
        fn = {"stream": stream_section, "match": match_section, "compose": compose_section,
              "batched": batched_section, "fwd_bwd": fwd_bwd_section, "c1": c1_section,
              "brackets": brackets_section, "compose_f32": compose_f32_section,
              "reduce_up_f32": reduce_up_f32_section,
              "small": lambda st, w: small_section(),
              "copy": lambda st, w: copy_ceiling(max(st, 1))}[args.only]
        print(json.dumps({args.only: fn(args.steps, args.warmup)}), flush=True)
        return

    import torch

    import gen
    import paper_2205_11659_amd as tb

    dev = torch.device("cuda:0")
    c = gen.config(2)
    n = len(c["kind"])
    kind = torch.from_numpy(c["kind"].view(np.int32)).to(dev)
    box = torch.from_numpy(c["box"]).to(dev)
    host = (c["kind"], c["box"]) if not args.no_cpu else None
    del c
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    match = torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)

    tuned = None
    if not args.no_tune:  # untimed: the autotuner picks the launch variant for this size
        tuned, _ = tb.tune_bbox(kind, box, reps=3)
    for _ in range(args.warmup):
        tb.tb_bbox(kind, box, match=match, out=out, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0, f"status {int(status.item())}"

    clocks_before = gpu_clocks()
    ev = HipEvents()
    pairs = [(ev.create(), ev.create()) for _ in range(args.steps)]
    # whole-step events on the stream the calls run on (torch's current one)
    steps_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        tb.lib().tb_profile_events(pairs[k][0], pairs[k][1])
        steps_ev[k][0].record()
        tb.tb_bbox(kind, box, match=match, out=out, status=status)
        steps_ev[k][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tb.lib().tb_profile_events(None, None)
    assert int(status.item()) == 0
    k_ms = float(np.mean([ev.elapsed_ms(a, b) for a, b in pairs]))
    ev_ms = np.array([a.elapsed_time(b) for a, b in steps_ev])
    clocks_after = gpu_clocks()

    ms_step = wall * 1e3 / args.steps
    med_ms = float(np.median(ev_ms))
    value = n / (med_ms / 1e3) / 1e9
    achieved = ALG_BYTES_FWD * n / (k_ms / 1e3) / 1e9
    res = {
        "metric": "Gelem/s + % HBM peak, match+bbox fwd(+bwd); batched vs per-scene launches",
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scene-128M-chain32M", "elements": n,
                   "structure": "chain of 2^25 alternating clip/blend opens around a cap-64 "
                                "random walk of 2^26 elements", "op": "tb_bbox forward"},
        "step_ms": {"median": round(med_ms, 4), "min": round(float(ev_ms.min()), 4),
                    "wall_mean": round(ms_step, 4),
                    "timing": "value from the median of per-step HIP events on the call's stream"},
        "path_hbm_frac": round(ALG_BYTES_FWD * n / (med_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "autotune": _tune_record(tuned) if tuned else None,
        "gpu_clocks": {"before": clocks_before, "after": clocks_after},
        "roofline": {"bound": "hbm", "kernel": "k_resolve", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "kernel_ms": round(k_ms, 4), "traffic": measured_traffic(),
                     "alg_bytes": ALG_BYTES_FWD * n},
    }
    if not args.no_extra:
        del kind, box, out, match
        torch.cuda.empty_cache()
        res["match_only"] = match_section(max(3, args.steps // 2), 2, host[0] if host else None)
        torch.cuda.empty_cache()
        res["compose"] = compose_section(max(3, args.steps // 2), 2, host[0] if host else None)
        torch.cuda.empty_cache()
        res["brackets"] = brackets_section(max(3, args.steps // 2), 2)
        res["compose_f32"] = compose_f32_section(max(3, args.steps // 2), 2)
        res["reduce_up_f32"] = reduce_up_f32_section(max(3, args.steps // 2), 2)
        res["stream"] = stream_section(max(3, args.steps // 2), 2)
        torch.cuda.empty_cache()
        res["batched_vs_per_scene"] = batched_section(max(3, args.steps // 2), 2, cpu=not args.no_cpu)
        res["fwd_bwd"] = fwd_bwd_section(max(3, args.steps // 2), 2)
        torch.cuda.empty_cache()
        res["c1"] = c1_section(max(3, args.steps // 2), 2)
        torch.cuda.empty_cache()
        res["small_scene"] = small_section()
        res["copy_ceiling"] = copy_ceiling()
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(*host)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
