// libtreebbox C ABI (include/treebbox.h): argument checks on the host, then
// the kernel pipelines.  No allocation happens here: the caller's workspace
// holds every intermediate array.
#include <hip/hip_runtime.h>

#include "../../include/treebbox.h"
#include "tb_forward.h"

namespace {

constexpr int64_t MAX_N = (int64_t)1 << 31;  // indices are int32

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t ws_bytes_for(int op, int64_t n, int64_t S) {
    if (n < 0 || n >= MAX_N) return 0;
    switch (op) {
    case TB_OP_MATCH:
    case TB_OP_BBOX:
        return tb::fwd_layout(n, 1, 16, false).total;
    case TB_OP_BBOX_BATCHED:
        if (S < 1 || S >= MAX_N) return 0;
        return tb::fwd_layout(n, S, 16, false).total;
    case TB_OP_BBOX_BACKWARD:
        return tb::fwd_layout(n, 1, 32, true).total;
    case TB_OP_COMPOSE:
        return tb::fwd_layout(n, 1, 24, false).total;
    case TB_OP_BBOX_STREAM:
        return tb::stream_layout(n).total;
    case TB_OP_COMPOSE_F32:
        return tb::compose_f32_layout(n).total;
    case TB_OP_REDUCE_UP_F32:
        return tb::reduce_up_layout(n).total;
    default:
        return 0;
    }
}

tb_status check_common(const void *kind, int64_t n, const void *ws, size_t ws_bytes, int op,
                       int64_t S) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!ws) return TB_ERR_NULL;
    if (n > 0 && !kind) return TB_ERR_NULL;
    if (!aligned(ws, 256) || (kind && !aligned(kind, 4))) return TB_ERR_ALIGN;
    size_t need = ws_bytes_for(op, n, S);
    if (need == 0 || ws_bytes < need) return TB_ERR_WORKSPACE;
    return TB_OK;
}

tb_status launched(hipError_t e) { return e == hipSuccess ? TB_OK : TB_ERR_HIP; }

}  // namespace

extern "C" {

size_t tb_workspace_bytes(int op, int64_t n, int64_t num_scenes) {
    return ws_bytes_for(op, n, num_scenes);
}

tb_status tb_match(const uint32_t *kind, int64_t n, int32_t *match, int32_t *pm, void *ws,
                   size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && !match)) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (match && !aligned(match, 4)) || (pm && !aligned(pm, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_MATCH, 1);
    if (c != TB_OK) return c;
    return launched(tb::fwd_run(false, kind, nullptr, n, nullptr, 1, match, pm, nullptr, ws,
                                dev_status, (hipStream_t)stream, tb::variant_for(TB_OP_MATCH, n, false)));
}

tb_status tb_match_brackets(const uint32_t *tok, int64_t n, int32_t *match, int32_t *pm, void *ws,
                            size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && !match)) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (match && !aligned(match, 4)) || (pm && !aligned(pm, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(tok, n, ws, ws_bytes, TB_OP_MATCH, 1);
    if (c != TB_OK) return c;
    return launched(tb::brackets_run(tok, n, match, pm, ws, dev_status, (hipStream_t)stream,
                                     tb::variant_for(TB_OP_MATCH, n, false)));
}

tb_status tb_bbox(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                  tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                  void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_BBOX, 1);
    if (c != TB_OK) return c;
    return launched(tb::fwd_run(true, kind, (const float4 *)box_in, n, nullptr, 1, match, nullptr,
                                (float4 *)box_out, ws, dev_status, (hipStream_t)stream,
                                tb::variant_for(TB_OP_BBOX, n, true)));
}

tb_status tb_compose(const uint32_t *kind, const tb_affine *xf_in, int64_t n, tb_affine *xf_out,
                     void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!xf_in || !xf_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (xf_in && !aligned(xf_in, 8)) || (xf_out && !aligned(xf_out, 8)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_COMPOSE, 1);
    if (c != TB_OK) return c;
    return launched(tb::compose_run(kind, xf_in, n, xf_out, ws, dev_status, (hipStream_t)stream));
}

tb_status tb_compose_f32(const uint32_t *kind, const float *xf_in, int64_t n, float *xf_out, void *ws,
                         size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!xf_in || !xf_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (xf_in && !aligned(xf_in, 8)) || (xf_out && !aligned(xf_out, 8)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_COMPOSE_F32, 1);
    if (c != TB_OK) return c;
    return launched(tb::compose_f32_run(kind, xf_in, n, xf_out, ws, dev_status, (hipStream_t)stream));
}

tb_status tb_reduce_up_f32(const uint32_t *kind, const float *xf_in, int64_t n, float *xf_out, void *ws,
                           size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!xf_in || !xf_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (xf_in && !aligned(xf_in, 8)) || (xf_out && !aligned(xf_out, 8)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_REDUCE_UP_F32, 1);
    if (c != TB_OK) return c;
    return launched(tb::reduce_up_run(kind, xf_in, n, xf_out, ws, dev_status, (hipStream_t)stream));
}

tb_status tb_bbox_stream(const uint32_t *tag, const tb_box *box_in, int64_t n, int32_t *match,
                         tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                         void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(tag, n, ws, ws_bytes, TB_OP_BBOX_STREAM, 1);
    if (c != TB_OK) return c;
    return launched(tb::stream_run(tag, (const float4 *)box_in, n, match, (float4 *)box_out, ws,
                                   dev_status, (hipStream_t)stream));
}

tb_status tb_bbox_batched(const uint32_t *kind, const tb_box *box_in, const int64_t *offsets,
                          int64_t num_scenes, int64_t total_n, int32_t *match, tb_box *box_out,
                          void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream) {
    if (total_n < 0 || total_n >= MAX_N || num_scenes < 1 || num_scenes >= MAX_N)
        return TB_ERR_SIZE;
    if (!dev_status || !offsets || (total_n > 0 && (!box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || !aligned(offsets, 8) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, total_n, ws, ws_bytes, TB_OP_BBOX_BATCHED, num_scenes);
    if (c != TB_OK) return c;
    return launched(tb::fwd_run(true, kind, (const float4 *)box_in, total_n, offsets, num_scenes,
                                match, nullptr, (float4 *)box_out, ws, dev_status,
                                (hipStream_t)stream, tb::variant_for(TB_OP_BBOX_BATCHED, total_n, true)));
}

tb_status tb_bbox_noalloc(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                          tb_box *box_out, uint32_t *dev_status, void *stream) {
    if (n < 0) return TB_ERR_SIZE;
    if (n > tb::NOALLOC_MAX_N) return TB_ERR_TOO_LARGE;
    if (!dev_status || (n > 0 && (!kind || !box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (kind && !aligned(kind, 4)) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    return launched(tb::fwd_run_noalloc(kind, (const float4 *)box_in, n, match, (float4 *)box_out,
                                        dev_status, (hipStream_t)stream));
}

tb_status tb_bbox_backward(const uint32_t *kind, const tb_box *box_in, const tb_box *grad_out,
                           int64_t n, tb_box *grad_in, void *ws, size_t ws_bytes,
                           uint32_t *dev_status, void *stream) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!box_in || !grad_out || !grad_in))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (box_in && !aligned(box_in, 16)) ||
        (grad_out && !aligned(grad_out, 16)) || (grad_in && !aligned(grad_in, 16)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_BBOX_BACKWARD, 1);
    if (c != TB_OK) return c;
    return launched(tb::bwd_run(kind, (const float4 *)box_in, (const float4 *)grad_out, n,
                                (float4 *)grad_in, ws, dev_status, (hipStream_t)stream));
}

// ---------------------------------------------------------------- tuning
static tb::Variant from_c(const tb_variant &v) { return tb::Variant{v.resolve_elems, v.reduce_elems, v.cross_records}; }
static tb_variant to_c(const tb::Variant &v) { return tb_variant{v.kr, v.kd, v.cu}; }

static tb_status tuned(hipError_t e, const tb::Variant &v, float best, float def, tb_variant *chosen,
                       float *ms) {
    if (e != hipSuccess) return TB_ERR_HIP;
    if (chosen) *chosen = to_c(v);
    if (ms) ms[0] = best, ms[1] = def;
    return TB_OK;
}

tb_status tb_tune_match(const uint32_t *kind, int64_t n, int32_t *match, int32_t *pm, void *ws,
                        size_t ws_bytes, uint32_t *dev_status, void *stream, int reps,
                        tb_variant *chosen, float *ms) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && !match)) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (match && !aligned(match, 4)) || (pm && !aligned(pm, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_MATCH, 1);
    if (c != TB_OK) return c;
    hipStream_t st = (hipStream_t)stream;
    tb::Variant v{};
    float best = 0, def = 0;
    hipError_t e = tb::tune(TB_OP_MATCH, n, false, reps, st, [&](tb::Variant var) {
        return tb::fwd_run(false, kind, nullptr, n, nullptr, 1, match, pm, nullptr, ws, dev_status, st, var);
    }, &v, &best, &def);
    return tuned(e, v, best, def, chosen, ms);
}

tb_status tb_tune_bbox(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                       tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                       void *stream, int reps, tb_variant *chosen, float *ms) {
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!dev_status || (n > 0 && (!box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, n, ws, ws_bytes, TB_OP_BBOX, 1);
    if (c != TB_OK) return c;
    hipStream_t st = (hipStream_t)stream;
    tb::Variant v{};
    float best = 0, def = 0;
    hipError_t e = tb::tune(TB_OP_BBOX, n, true, reps, st, [&](tb::Variant var) {
        return tb::fwd_run(true, kind, (const float4 *)box_in, n, nullptr, 1, match, nullptr,
                           (float4 *)box_out, ws, dev_status, st, var);
    }, &v, &best, &def);
    return tuned(e, v, best, def, chosen, ms);
}

tb_status tb_tune_bbox_batched(const uint32_t *kind, const tb_box *box_in, const int64_t *offsets,
                               int64_t num_scenes, int64_t total_n, int32_t *match, tb_box *box_out,
                               void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream,
                               int reps, tb_variant *chosen, float *ms) {
    if (total_n < 0 || total_n >= MAX_N || num_scenes < 1 || num_scenes >= MAX_N)
        return TB_ERR_SIZE;
    if (!dev_status || !offsets || (total_n > 0 && (!box_in || !box_out))) return TB_ERR_NULL;
    if (!aligned(dev_status, 4) || !aligned(offsets, 8) || (box_in && !aligned(box_in, 16)) ||
        (box_out && !aligned(box_out, 16)) || (match && !aligned(match, 4)))
        return TB_ERR_ALIGN;
    tb_status c = check_common(kind, total_n, ws, ws_bytes, TB_OP_BBOX_BATCHED, num_scenes);
    if (c != TB_OK) return c;
    hipStream_t st = (hipStream_t)stream;
    tb::Variant v{};
    float best = 0, def = 0;
    hipError_t e = tb::tune(TB_OP_BBOX_BATCHED, total_n, true, reps, st, [&](tb::Variant var) {
        return tb::fwd_run(true, kind, (const float4 *)box_in, total_n, offsets, num_scenes, match,
                           nullptr, (float4 *)box_out, ws, dev_status, st, var);
    }, &v, &best, &def);
    return tuned(e, v, best, def, chosen, ms);
}

static bool tunable_op(int op) { return op == TB_OP_MATCH || op == TB_OP_BBOX || op == TB_OP_BBOX_BATCHED; }

tb_status tb_variant_get(int op, int64_t n, tb_variant *out) {
    if (!tunable_op(op)) return TB_ERR_ARG;
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (!out) return TB_ERR_NULL;
    *out = to_c(tb::variant_for(op, n, op != TB_OP_MATCH));
    return TB_OK;
}

tb_status tb_variant_set(int op, int64_t n, const tb_variant *v) {
    if (!tunable_op(op)) return TB_ERR_ARG;
    if (n < 0 || n >= MAX_N) return TB_ERR_SIZE;
    if (v) {
        const tb::Variant x = from_c(*v);
        if (!tb::variant_ok(x) || (op == TB_OP_MATCH && x.cu != 4)) return TB_ERR_ARG;
        tb::variant_set(op, n, &x);
    } else {
        tb::variant_set(op, n, nullptr);
    }
    return TB_OK;
}

tb_status tb_tune_save(const char *path) {
    if (!path) return TB_ERR_NULL;
    return tb::tune_save(path) ? TB_OK : TB_ERR_ARG;
}

tb_status tb_tune_load(const char *path) {
    if (!path) return TB_ERR_NULL;
    return tb::tune_load(path) ? TB_OK : TB_ERR_ARG;
}

void tb_tune_clear(void) { tb::tune_clear(); }

void tb_profile_events(void *before, void *after) {
    tb::g_prof_before = (hipEvent_t)before;
    tb::g_prof_after = (hipEvent_t)after;
}

const char *tb_status_str(tb_status s) {
    switch (s) {
    case TB_OK: return "TB_OK";
    case TB_ERR_NULL: return "TB_ERR_NULL: a required pointer is NULL";
    case TB_ERR_SIZE: return "TB_ERR_SIZE: size out of range";
    case TB_ERR_ALIGN: return "TB_ERR_ALIGN: misaligned pointer";
    case TB_ERR_WORKSPACE: return "TB_ERR_WORKSPACE: workspace too small";
    case TB_ERR_ARG: return "TB_ERR_ARG: invalid argument";
    case TB_ERR_HIP: return "TB_ERR_HIP: HIP launch failed";
    case TB_ERR_TOO_LARGE:
        return "TB_ERR_TOO_LARGE: n exceeds the no-allocation variant's maximum of 2^20 elements";
    }
    return "unknown tb_status";
}

}  // extern "C"
