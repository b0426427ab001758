// Host-side entry into the forward kernels (tb_forward.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <vector>

namespace tb {

// Byte offsets of the forward pipeline's arrays inside the caller's workspace.
struct FwdLayout {
    int64_t M, Mp, nb;
    int levels;
    size_t pinfo, part, mtree, bagg, crbase, crtot, jptr0, jptr1, jval0, jval1;
    size_t U_idx, U_cum, U_suf, cr_slot, cr_c, cr_pre;
    size_t runs, rhead, ptot, upre, usuf, sp, spb, status, offflag, acc, selfm;
    size_t total;
};

// vbytes: payload size (16 forward, 32 backward); grad adds the gradient
// accumulators.
FwdLayout fwd_layout(int64_t n, int64_t S, size_t vbytes, bool grad);

// Launch shape of one forward call: elements per thread of the main pass
// (kr) and of the reduce pass (kd), 4 or 8, and close records per thread of
// the cross-partition pass (cu: 2, 4 or 8).  Partitions stay T elements, so
// the workspace does not depend on the variant.
struct Variant {
    int kr = 0, kd = 0, cu = 0;
};
inline bool variant_ok(const Variant &v) {
    return (v.kr == 4 || v.kr == 8) && (v.kd == 4 || v.kd == 8) && (v.cu == 2 || v.cu == 4 || v.cu == 8);
}
inline Variant default_variant(bool boxes) {
    // matching alone needs few registers: 8 elements per thread halve the
    // per-thread share of the partition-level steps
    return boxes ? Variant{4, 4, 4} : Variant{8, 8, 4};
}

// Enqueue the forward pipeline.  boxes=false computes matching only.
// off == nullptr means one scene.  status may be nullptr (workspace word).
// An invalid variant means the default one.
hipError_t fwd_run(bool boxes, const uint32_t *kind, const float4 *box, int64_t n,
                   const int64_t *off, int64_t S, int32_t *match, int32_t *pm, float4 *out,
                   void *ws, uint32_t *status, hipStream_t st, Variant var);

// Matching over typed bracket tokens (0 none, 2t+1 open type t, 2t+2 close
// type t): a close whose type differs from its open's sets KIND_MISMATCH.
hipError_t brackets_run(const uint32_t *tok, int64_t n, int32_t *match, int32_t *pm, void *ws,
                        uint32_t *status, hipStream_t st, Variant var);

// Transform composition down the tree: xf and out hold 24-byte rows
// [a b c d e f] (uint32, 8-byte aligned).
hipError_t compose_run(const uint32_t *kind, const void *xf, int64_t n, void *out, void *ws,
                       uint32_t *status, hipStream_t st);

// fp32 transforms composed down the tree in pointer-jumping order: the
// matching workspace, then pm, two pointer and two value buffers, flags.
struct ComposeF32Layout {
    FwdLayout f;
    size_t pm, ptr0, ptr1, val0, val1, flags;
    size_t total;
};
ComposeF32Layout compose_f32_layout(int64_t n);
hipError_t compose_f32_run(const uint32_t *kind, const float *xf, int64_t n, float *out, void *ws,
                           uint32_t *status, hipStream_t st);

// fp32 transforms of the leaves multiplied up the tree (segment-tree
// grouping): the matching workspace, the partners, the 2N tree nodes.
struct ReduceUpLayout {
    FwdLayout f;
    int64_t N;
    size_t match, node;
    size_t total;
};
ReduceUpLayout reduce_up_layout(int64_t n);
hipError_t reduce_up_run(const uint32_t *kind, const float *xf, int64_t n, float *out, void *ws,
                         uint32_t *status, hipStream_t st);

// Draw-object stream front end: the forward pipeline's workspace for n
// elements (the extracted count is at most n), then the extracted arrays.
struct StreamLayout {
    FwdLayout f;
    int64_t nblk;
    size_t ckind, cbox, cidx, cmatch, cnt, m;
    size_t total;
};
StreamLayout stream_layout(int64_t n);

// Extract the tree elements of a tag stream (tag 5: outside the tree), run
// the forward pipeline on them, write rows and partners at stream positions.
hipError_t stream_run(const uint32_t *tag, const float4 *box, int64_t n, int32_t *match,
                      float4 *out, void *ws, uint32_t *status, hipStream_t st);

// Enqueue the gradient pass (recompute with attaining indices + exact sums).
hipError_t bwd_run(const uint32_t *kind, const float4 *box, const float4 *grad_out, int64_t n,
                   float4 *grad_in, void *ws, uint32_t *status, hipStream_t st);

// tb_bbox over a fixed per-device array instead of a caller's workspace
// (no allocation anywhere).  NOALLOC_MAX_N elements at most: their forward
// workspace fits in NOALLOC_BYTES.
constexpr int64_t NOALLOC_MAX_N = (int64_t)1 << 20;
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
hipError_t fwd_run_noalloc(const uint32_t *kind, const float4 *box, int64_t n, int32_t *match,
                           float4 *out, uint32_t *status, hipStream_t st);

// Autotuner (tb_tune.cpp): the variant that calls of `op` on n elements use
// on the current device (the default until tuned or set), and the timing of
// every candidate on a caller's input.  `call` runs one whole forward call
// with the given variant on the stream.
Variant variant_for(int op, int64_t n, bool boxes);
void variant_set(int op, int64_t n, const Variant *v);  // nullptr: back to the default
std::vector<Variant> candidates(bool boxes);
hipError_t tune(int op, int64_t n, bool boxes, int reps, hipStream_t st,
                const std::function<hipError_t(Variant)> &call, Variant *chosen, float *best_ms,
                float *default_ms);
bool tune_save(const char *path);
bool tune_load(const char *path);
void tune_clear();

// Events recorded around the main per-partition kernel (nullptr = off).
extern hipEvent_t g_prof_before, g_prof_after;

}  // namespace tb
