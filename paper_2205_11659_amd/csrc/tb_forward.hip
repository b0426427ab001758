// libtreebbox forward kernels: parentheses matching, clip intersections and
// blend unions over a flattened scene tree (arXiv 2205.11659), for gfx950.
//
// Pipeline (one call):
//   k_reduce      per partition of T elements: partition stack summary --
//                 pops of the incoming stack (a), surviving unmatched opens
//                 (index + clip intersection of the surviving opens up to
//                 each one), scene-reset flag.  Reads kinds only, plus the
//                 boxes of surviving clip opens.  This is the paper's "stack
//                 slice" (section "Simple GPU parentheses matching
//                 algorithm", Stack slices; boxes per section "GPU
//                 implementation of clipping and blending").
//   k_spine_scan  segmented depth scan over partitions; min tree of the
//                 partitions' lowest levels.
//   k_spine_link  owner link of each partition: the nearest earlier
//                 partition whose lowest level is smaller (it holds the
//                 stack entry just below); seeds pointer jumping.
//   k_jump        pointer jumping along owner links: the clip context at
//                 each partition's base level (the paper's pointer jumping,
//                 section "Parallel bounding boxes", Clips, applied to
//                 partitions instead of elements).
//   k_resolve     per partition: reads kinds and boxes once, rebuilds the
//                 incoming stack levels it pops (suffix relation, section
//                 "The stack monoid"), resolves matches, clips and blend
//                 unions inside the partition, and leaves records for blends
//                 whose open lies in an earlier partition.
//   k_ublocks / k_usparse   range-union structure over partition totals.
//   k_cross       finishes blends that span partitions: the union of the
//                 open's suffix, the whole partitions between, and the
//                 close's prefix, written at both rows (the union stored at
//                 the open as well as the close, last paragraph of "GPU
//                 implementation of clipping and blending").
#include "tb_common.h"
#include "tb_forward.h"

namespace tb {

// ------------------------------------------------------------------ utils
__global__ void k_zero_u32(uint32_t *p, int64_t cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0u;
}

// offsets must satisfy 0 = o[0] <= o[1] <= ... <= o[S] = n
__global__ void k_check_offsets(const int64_t *off, int64_t S, int64_t n, uint32_t *status) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S) return;
    bool bad = (s == 0 && off[0] != 0) || (s == S && off[S] != n) || (s < S && off[s] > off[s + 1]);
    if (bad)
        for (int64_t q = 0; q < S; ++q) atomicOr(status + q, ST_BAD_OFF);
}

// ---------------------------------------------------------------- k_reduce
template <bool BOXES>
__global__ __launch_bounds__(W) void k_reduce(const uint32_t *__restrict__ kind,
                                              const float4 *__restrict__ box, int64_t n,
                                              const int64_t *__restrict__ off, int64_t S,
                                              int4 *__restrict__ pinfo,
                                              int32_t *__restrict__ U_idx,
                                              float4 *__restrict__ U_cum) {
    __shared__ Seg sh_seg[NWAVE];
    __shared__ int sh_i[NWAVE];
    __shared__ Box sh_b[NWAVE];
    __shared__ int mt[2 * W];
    const int t = threadIdx.x;
    const int64_t P = blockIdx.x;
    const int64_t g0 = P * T + (int64_t)t * K;

    uint32_t ks[K];
    load_kinds(kind, n, g0, ks);
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (ks[j] > 4u) ks[j] = LEAF;
    const uint32_t rm = reset_mask(off, S, g0);
    const Walk wk = walk_kinds(ks, rm);
    const int b = __popc(wk.umask);

    Seg tot;
    const Seg ex = block_excl_scan<NWAVE>(Seg{wk.rs ? 1 : 0, wk.rs ? b : b - wk.a}, SegOp{},
                                          Seg{0, 0}, sh_seg, &tot);
    const int D = ex.v;  // depth at thread start: partition-relative unless ex.r
    const int cm = wk.rs ? SENT : D - wk.a;
    const int base = wk.rs ? 0 : D - wk.a;
    // pops below the partition start happen only before the first reset
    int lo_tot;
    block_excl_scan<NWAVE>(ex.r ? INT32_MAX : D - wk.a, MinOp{}, INT32_MAX, sh_i, &lo_tot);
    const int aP = lo_tot < 0 ? -lo_tot : 0;
    int rcount;
    block_excl_scan<NWAVE>(wk.rs ? 1 : 0, AddOp{}, 0, sh_i, &rcount);
    const bool rP = rcount > 0;
    const int baseP = rP ? 0 : -aP;

    // an unmatched open at level L survives the partition unless a later
    // thread's lowest level is below L
    mintree_build(mt, cm);
    const int sufmin = mintree_range_min(mt, t + 1, W - 1);
    int ns = 0;
    if ((int64_t)sufmin > (int64_t)base) ns = (int)min((int64_t)b, (int64_t)sufmin - base);

    Box agg = box_inf(), bxs[K];
    uint32_t clipmask = 0;
    if (BOXES) {
        int jj = 0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            bxs[p] = box_inf();
            if ((wk.umask >> p) & 1u) {
                if (jj < ns && ks[p] == BCLIP) {
                    bxs[p] = ld_box(box, g0 + p);
                    agg = isect(agg, bxs[p]);
                    clipmask |= 1u << p;
                }
                ++jj;
            }
        }
    }
    Box aggtot;
    Box cum = BOXES ? block_excl_scan<NWAVE>(agg, IsectOp{}, box_inf(), sh_b, &aggtot) : box_inf();
    int nsum;
    block_excl_scan<NWAVE>(ns, AddOp{}, 0, sh_i, &nsum);

    int jj = 0;
#pragma unroll
    for (int p = 0; p < K; ++p) {
        if (!((wk.umask >> p) & 1u)) continue;
        if (jj < ns) {
            const int64_t L = (int64_t)base + 1 + jj;
            const int64_t slot = L - baseP - 1;
            if (slot >= 0 && slot < T) {
                U_idx[P * T + slot] = (int32_t)((uint32_t)(g0 + p) | (ks[p] == BBLEND ? BLEND_BIT : 0u));
                if (BOXES) {
                    if ((clipmask >> p) & 1u) cum = isect(cum, bxs[p]);
                    st_box(U_cum, P * T + slot, cum);
                }
            }
        }
        ++jj;
    }
    if (t == 0) pinfo[P] = make_int4(aP, nsum, rP ? 1 : 0, 0);
}

// ------------------------------------------------------------ spine kernels
// One workgroup of SPW threads: segmented exclusive depth scan over the M
// partition summaries, partition records {d, cm, base, link}, the min tree
// over cm, and the end-of-sequence balance check.
constexpr int SPW = 1024;

__global__ __launch_bounds__(SPW) void k_spine_scan(const int4 *__restrict__ pinfo, int64_t M,
                                                     int4 *__restrict__ part, int *__restrict__ mtree,
                                                     int64_t Mp, const int64_t *__restrict__ off,
                                                     int64_t S, int64_t n,
                                                     uint32_t *__restrict__ status) {
    __shared__ Seg sh_seg[SPW / WAVE];
    const int t = threadIdx.x;
    const int64_t ipt = (M + SPW - 1) / SPW;
    const int64_t lo = t * ipt, hi = min(M, lo + ipt);
    Seg agg{0, 0};
    for (int64_t P = lo; P < hi; ++P) {
        int4 v = pinfo[P];
        agg = SegOp{}(agg, Seg{v.z, v.z ? v.y : v.y - v.x});
    }
    Seg tot;
    Seg ex = block_excl_scan<SPW / WAVE>(agg, SegOp{}, Seg{0, 0}, sh_seg, &tot);
    int d = ex.v;
    for (int64_t P = lo; P < hi; ++P) {
        int4 v = pinfo[P];
        const int pre_m = d - v.x;
        const int cm = v.z ? SENT : pre_m;
        part[P] = make_int4(d, cm, v.z ? 0 : pre_m, -1);
        mtree[Mp + P] = cm;
        d = v.z ? v.y : d - v.x + v.y;
    }
    for (int64_t P = M + t; P < Mp; P += SPW) mtree[Mp + P] = INT32_MAX;
    if (t == 0 && tot.v != 0 && n > 0) flag(status, off, S, n - 1, ST_UNBAL);
    __syncthreads();
    for (int64_t w = Mp / 2; w >= 1; w >>= 1) {
        for (int64_t x = w + t; x < 2 * w; x += SPW) {
            int a = mtree[2 * x], b = mtree[2 * x + 1];
            mtree[x] = a < b ? a : b;
        }
        __syncthreads();
    }
}

// rightmost partition Q < P with cm[Q] < v over the global min tree, or -1
__device__ __forceinline__ int64_t gtree_prev_less(const int *mt, int64_t Mp, int64_t P, int64_t v) {
    int64_t x = Mp + P;
    while (x > 1) {
        if ((x & 1) && (int64_t)mt[x - 1] < v) {
            x = x - 1;
            while (x < Mp) x = ((int64_t)mt[2 * x + 1] < v) ? 2 * x + 1 : 2 * x;
            return x - Mp;
        }
        x >>= 1;
    }
    return -1;
}

template <bool BOXES>
__global__ void k_spine_link(const int4 *__restrict__ pinfo, int4 *__restrict__ part, int64_t M,
                             const int *__restrict__ mtree, int64_t Mp,
                             const float4 *__restrict__ U_cum, int32_t *__restrict__ jptr,
                             float4 *__restrict__ jval) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M) return;
    int4 pr = part[P];
    const int64_t cm = pr.y;
    int64_t link = -1;
    if (cm != SENT) link = gtree_prev_less(mtree, Mp, P, cm);
    part[P].w = (int)link;
    if (!BOXES) return;
    Box val = box_inf();
    int64_t ptr = -1;
    if (cm != SENT && cm > 0 && link >= 0) {
        const int64_t slot = cm - (int64_t)part[link].z - 1;
        if (slot >= 0 && slot < pinfo[link].y) {
            val = ld_box(U_cum, link * T + slot);
            ptr = link;
        }
    }
    jptr[P] = (int32_t)ptr;
    st_box(jval, P, val);
}

__global__ void k_jump(const int32_t *__restrict__ ptr_in, const float4 *__restrict__ val_in,
                       int32_t *__restrict__ ptr_out, float4 *__restrict__ val_out, int64_t M) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M) return;
    int32_t p = ptr_in[P];
    Box v = ld_box(val_in, P);
    if (p >= 0) {
        v = isect(v, ld_box(val_in, p));
        p = ptr_in[p];
    }
    ptr_out[P] = p;
    st_box(val_out, P, v);
}

// ---------------------------------------------------------------- k_runs
// Owner runs of each partition's incoming levels [max(preM,1), dP]: walking
// the owner links from P-1, each owner R holds a contiguous range of levels
// (its surviving opens).  One thread per partition; many chains are walked
// at once, which hides the dependent loads.  Up to RMAX runs are stored;
// head = {count, next owner, next top level, complete}.
__global__ void k_runs(const int4 *__restrict__ pinfo, const int4 *__restrict__ part, int64_t M,
                       int4 *__restrict__ runs, int4 *__restrict__ rhead) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M) return;
    const int64_t dP = part[P].x;
    const int64_t preM = dP - pinfo[P].x;
    const int64_t need_lo = preM > 1 ? preM : 1;
    int64_t R = P - 1, hi = dP;
    int nr = 0;
    while (nr < RMAX && R >= 0 && hi >= need_lo) {
        const int4 pr = part[R];
        const int64_t from = max((int64_t)pr.z + 1, need_lo);
        if (from <= hi) runs[P * RMAX + nr++] = make_int4((int)R, (int)from, (int)hi, pr.z);
        if (pr.y == SENT) {
            R = -1;
            break;
        }
        hi = min(hi, (int64_t)pr.y);
        R = pr.w;
    }
    const bool complete = !(R >= 0 && hi >= need_lo);
    rhead[P] = make_int4(nr, (int)R, (int)hi, complete ? 1 : 0);
}

// ------------------------------------------------------------- k_resolve
// Stack entry at some level as seen from the start of a thread.
struct Ent {
    int64_t idx;  // element index of the open, -1 = root
    Box ctx;      // clip context of the entry (its children's context)
    int kind;     // kind of the open (BCLIP/BBLEND), -1 for root
    int own;      // owning thread in this partition, or -1
    int pos;      // position of the open in the owning thread
    int slot;     // global U slot when owned by an earlier partition, else -1
};

__device__ __forceinline__ Ent ent_root() { return Ent{-1, box_inf(), -1, -1, -1, -1}; }

// Owner run holding level L (runs cover disjoint level ranges, highest
// first): binary search; -1 if L lies below the stored runs.
__device__ __forceinline__ int find_run(const int4 *runs, int nruns, int64_t L) {
    int lo = 0, hi = nruns - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int4 r = runs[mid];
        if (L > r.z)
            hi = mid - 1;
        else if (L < r.y)
            lo = mid + 1;
        else
            return mid;
    }
    return -1;
}

// Slot of the entry at level L >= 1 held by an earlier partition (global U
// slot), or -1.  Continues the owner walk when the stored runs end early.
__device__ int64_t incoming_slot(int64_t L, const int4 *runs, int nruns, int4 head,
                                 const int4 *__restrict__ part, int64_t *owner) {
    int64_t R = -1, base = 0;
    const int r = find_run(runs, nruns, L);
    if (r >= 0) {
        R = runs[r].x;
        base = runs[r].w;
    } else if (!head.w) {
        int64_t RR = head.y, hi = head.z;
        while (RR >= 0 && hi >= L) {
            const int4 pr = part[RR];
            if (L > pr.z && L <= hi) {
                R = RR;
                base = pr.z;
                break;
            }
            if (pr.y == SENT) break;
            hi = min(hi, (int64_t)pr.y);
            RR = pr.w;
        }
    }
    *owner = R;
    if (R < 0 || L - base - 1 < 0 || L - base - 1 >= T) return -1;
    return R * T + (L - base - 1);
}

template <bool BOXES>
struct ResolveSmem {
    int4 runs[RMAX];
    // incoming levels [preM, dP], entry x = level preM + x: the open's index
    // (| BLEND_BIT) or -1 for the root, and its clip context.  After the walk
    // the context array is reused as the union tree over threads.
    int inc_idx[T + 1];
    Box inc_ctx[BOXES ? T + 1 : 1];
    Box ucum[BOXES ? T : 1];  // local clip prefix of thread U entries; later suffix unions
    Box jval[BOXES ? W : 1];  // clip context at each thread's base level
    uint8_t tkind[T];
    int tcm[W];
    int tbase[W];
    uint8_t tum[W];
    int mt[2 * W];
    int jptr[W];
    Seg sh_seg[NWAVE];
};

template <bool BOXES>
__global__ __launch_bounds__(W) void k_resolve(
    const uint32_t *__restrict__ kind, const float4 *__restrict__ box, int64_t n,
    const int64_t *__restrict__ off, int64_t S, const int4 *__restrict__ pinfo,
    const int4 *__restrict__ part, const int4 *__restrict__ runs_g,
    const int4 *__restrict__ rhead_g, const float4 *__restrict__ base_ctx,
    const int32_t *__restrict__ U_idx, const float4 *__restrict__ U_cum,
    float4 *__restrict__ U_suf, int32_t *__restrict__ cr_slot, int32_t *__restrict__ cr_c,
    float4 *__restrict__ cr_pre, float4 *__restrict__ ptot, int32_t *__restrict__ match,
    int32_t *__restrict__ pm, float4 *__restrict__ out, uint32_t *__restrict__ status) {
    __shared__ ResolveSmem<BOXES> sm;
    Box *ut = sm.inc_ctx;  // valid once the walk is over
    const int t = threadIdx.x, lane = t & (WAVE - 1), wbase = t & ~(WAVE - 1);
    const int64_t P = blockIdx.x;
    const int64_t p0 = P * T;
    const int64_t g0 = p0 + (int64_t)t * K;
    const int4 myp = part[P];
    const int64_t dP = myp.x;
    const int aP = pinfo[P].x;
    const int64_t preM = dP - aP;  // lowest incoming level any element here can see
    const int4 head = rhead_g[P];
    const int nruns = head.x;

    // ---- loads: inputs, owner runs
    uint32_t kr[K], ks[K];
    load_kinds(kind, n, g0, kr);
    Box bx[K];
    if (BOXES) {
#pragma unroll
        for (int j = 0; j < K; ++j) bx[j] = (g0 + j < n) ? ld_box(box, g0 + j) : box_empty();
    }
    if (t < RMAX) sm.runs[t] = runs_g[P * RMAX + t];
#pragma unroll
    for (int j = 0; j < K; ++j) ks[j] = kr[j] > 4u ? LEAF : kr[j];
    const uint32_t rm = reset_mask(off, S, g0);
    __syncthreads();

    // ---- gather the incoming levels [preM, dP] (issued now, stored later)
    constexpr int NG = (T + W) / W;  // entries per thread
    int g_idx[NG];
    Box g_ctx[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        g_idx[q] = -1;
        g_ctx[q] = box_inf();
        const int x = t + q * W;
        const int64_t L = preM + x;
        if (x > aP || L < 1) continue;
        int64_t R;
        const int64_t slot = incoming_slot(L, sm.runs, nruns, head, part, &R);
        if (slot < 0) continue;
        g_idx[q] = U_idx[slot];
        if (BOXES) g_ctx[q] = isect(ld_box(U_cum, slot), ld_box(base_ctx, R));
    }

    // ---- per-thread walk and thread-level depths
    const Walk wk = walk_kinds(ks, rm);
    const int b = __popc(wk.umask);
    Seg segtot;
    const Seg ex = block_excl_scan<NWAVE>(Seg{wk.rs ? 1 : 0, wk.rs ? b : b - wk.a}, SegOp{},
                                          Seg{0, 0}, sm.sh_seg, &segtot);
    const int64_t Dt = ex.r ? (int64_t)ex.v : dP + ex.v;  // absolute depth at thread start
    const int64_t pre_m = Dt - wk.a;
    const int cm = wk.rs ? SENT : (int)pre_m;
    const int base = wk.rs ? 0 : (int)pre_m;
    sm.tcm[t] = cm;
    sm.tbase[t] = base;
    sm.tum[t] = (uint8_t)wk.umask;
#pragma unroll
    for (int j = 0; j < K; ++j) sm.tkind[t * K + j] = (uint8_t)ks[j];
    if (BOXES) {
        Box c = box_inf();
#pragma unroll
        for (int p = 0; p < K; ++p) {
            if ((wk.umask >> p) & 1u) {
                if (ks[p] == BCLIP) c = isect(c, bx[p]);
                sm.ucum[t * K + p] = c;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const int x = t + q * W;
        if (x > aP) continue;
        sm.inc_idx[x] = g_idx[q];
        if (BOXES) sm.inc_ctx[x] = g_ctx[q];
    }
    mintree_build(sm.mt, cm);  // its barriers also publish everything above

    // levels at or below `lowtop` are held by no earlier thread of this
    // partition: they come from earlier partitions (the LDS table).
    const int64_t lowtop = min((int64_t)mintree_range_min(sm.mt, 0, t - 1), Dt);

    // ---- clip context at each thread's base level: pointer jumping along
    // owner threads, first inside the wave with shuffles, then across waves.
    if (BOXES) {
        Box v = box_inf();
        int ptr = -1;
        if (!wk.rs && pre_m > 0) {
            const int s = mintree_prev_less(sm.mt, t, pre_m);
            if (s >= 0) {
                const int64_t jj = pre_m - sm.tbase[s] - 1;
                const uint32_t um = sm.tum[s];
                if (jj >= 0 && jj < __popc(um)) {
                    v = sm.ucum[s * K + nth_bit(um, (int)jj)];
                    ptr = s;
                }
            } else {
                const int64_t x = pre_m - preM;
                if (x >= 0 && x <= aP) v = sm.inc_ctx[x];
            }
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const bool in = ptr >= wbase;
            const int src = in ? ptr - wbase : lane;
            const Box vv = {__shfl(v.x0, src, WAVE), __shfl(v.y0, src, WAVE), __shfl(v.x1, src, WAVE),
                            __shfl(v.y1, src, WAVE)};
            const int pp = __shfl(ptr, src, WAVE);
            if (in) {
                v = isect(v, vv);
                ptr = pp;
            }
        }
        sm.jval[t] = v;
        sm.jptr[t] = ptr;
        for (int r = 0; r < NWAVE && __syncthreads_or(ptr >= 0); ++r) {
            if (ptr >= 0) {
                v = isect(v, sm.jval[ptr]);
                ptr = sm.jptr[ptr];
            }
            __syncthreads();
            sm.jval[t] = v;
            sm.jptr[t] = ptr;
        }
        __syncthreads();
    }

    // ---- sequential walk over this thread's elements with a register stack
    // of local opens (index 0 = top; pushes and pops shift), each entry with
    // its clip context and the union of leaves seen since it was opened.
    int64_t sid = off ? scene_of(off, S, g0) : 0;
    int64_t soff = off ? off[sid] : 0;
    uint32_t defmask = 0;
    int depth = 0;  // local stack depth
    bool rseen = false;
    int64_t dep = Dt;
    int st_pos[K], st_kind[K];
    Box st_ctx[K], st_acc[K], lout[K];
    int def_own[K], def_pos[K];
    int64_t def_L[K];
    // the stack entry at level `cur_L` seen from this thread's start
    int64_t cur_L = INT64_MIN, cur_idx = -1;
    int cur_kind = -1, cur_own = -1, cur_pos = -1;
    Box cur_ctx = box_inf();
#pragma unroll
    for (int j = 0; j < K; ++j) {
        st_pos[j] = 0;
        st_kind[j] = 0;
        st_ctx[j] = box_inf();
        st_acc[j] = box_empty();
        lout[j] = box_empty();
        def_own[j] = def_pos[j] = -1;
        def_L[j] = 0;
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < K; ++j) {
        const int64_t i = g0 + j;
        const bool real = i < n;
        if ((rm >> j) & 1u) {
            if (real && i > 0 && dep != 0) flag(status, off, S, i - 1, ST_UNBAL);
            depth = 0;
            rseen = true;
            dep = 0;
            if (off && real) {
                sid = scene_of(off, S, i);
                soff = off[sid];
            }
        }
        if (real && kr[j] > 4u) flag(status, off, S, i, ST_BAD_KIND);
        if (depth == 0 && !rseen && cur_L != dep) {
            cur_L = dep;
            cur_idx = -1;
            cur_kind = -1;
            cur_own = -1;
            cur_ctx = box_inf();
            if (dep >= 1 && dep <= lowtop) {
                const int64_t x = dep - preM;
                if (x >= 0 && x <= aP) {
                    const int u = sm.inc_idx[x];
                    if (u != -1) {
                        cur_idx = (int64_t)((uint32_t)u & ~BLEND_BIT);
                        cur_kind = ((uint32_t)u & BLEND_BIT) ? (int)BBLEND : (int)BCLIP;
                        if (BOXES) cur_ctx = sm.inc_ctx[x];
                    }
                }
            } else if (dep > lowtop) {
                const int s = mintree_prev_less(sm.mt, t, dep);
                if (s >= 0) {
                    const int64_t jj = dep - sm.tbase[s] - 1;
                    const uint32_t um = sm.tum[s];
                    if (jj >= 0 && jj < __popc(um)) {
                        const int p = nth_bit(um, (int)jj);
                        cur_idx = p0 + (int64_t)s * K + p;
                        if (BOXES) cur_ctx = isect(sm.jval[s], sm.ucum[s * K + p]);
                        cur_kind = sm.tkind[s * K + p];
                        cur_own = s;
                        cur_pos = p;
                    }
                }
            }
        }
        int64_t top;
        Box ctx;
        if (depth > 0) {
            top = g0 + st_pos[0];
            ctx = st_ctx[0];
        } else if (rseen) {
            top = -1;
            ctx = box_inf();
        } else {
            top = cur_idx;
            ctx = cur_ctx;
        }
        if (pm && real) pm[i] = top >= 0 ? (int32_t)(top - soff) : -1;
        const uint32_t k = ks[j];
        if (k == LEAF) {
            if (BOXES) {
                const Box o = canon(isect(bx[j], ctx));
                lout[j] = o;
                st_acc[0] = unite(st_acc[0], o);  // harmless when the stack is empty
                if (real) st_box(out, i, o);
            }
            if (match && real) match[i] = -1;
        } else if (is_open(k)) {
            Box c = ctx;
            if (k == BCLIP) {
                c = isect(bx[j], ctx);
                if (BOXES && real) st_box(out, i, canon(c));
            }
#pragma unroll
            for (int q = K - 1; q > 0; --q) {
                st_pos[q] = st_pos[q - 1];
                st_kind[q] = st_kind[q - 1];
                st_ctx[q] = st_ctx[q - 1];
                st_acc[q] = st_acc[q - 1];
            }
            st_pos[0] = j;
            st_kind[0] = (int)k;
            st_ctx[0] = c;
            st_acc[0] = box_empty();
            ++depth;
            ++dep;
        } else if (depth > 0) {  // close matched inside this thread
            const int p = st_pos[0];
            const int ko = st_kind[0];
            const Box oc = st_ctx[0];
            const Box acc = st_acc[0];
#pragma unroll
            for (int q = 0; q < K - 1; ++q) {
                st_pos[q] = st_pos[q + 1];
                st_kind[q] = st_kind[q + 1];
                st_ctx[q] = st_ctx[q + 1];
                st_acc[q] = st_acc[q + 1];
            }
            st_acc[0] = unite(st_acc[0], acc);  // leaves flow up to the new top
            --depth;
            --dep;
            if ((k == ECLIP) != (ko == (int)BCLIP) && real) flag(status, off, S, i, ST_MISMATCH);
            if (match && real) {
                match[i] = (int32_t)(g0 + p - soff);
                match[g0 + p] = (int32_t)(i - soff);
            }
            if (BOXES && real) {
                if (k == ECLIP) {
                    st_box(out, i, canon(oc));
                } else {
                    st_box(out, i, acc);
                    st_box(out, g0 + p, acc);
                }
            }
        } else if (rseen) {  // close below its scene's root
            if (real) flag(status, off, S, i, ST_UNBAL);
        } else {  // close of the open at level `dep`, held before this thread
            const int64_t L = dep;
            if (L <= 0 || cur_idx < 0) {
                if (real) flag(status, off, S, i, ST_UNBAL);
            } else {
                if (((k == ECLIP) != (cur_kind == (int)BCLIP)) && real)
                    flag(status, off, S, i, ST_MISMATCH);
                if (match && real) {
                    match[i] = (int32_t)(cur_idx - soff);
                    if (cur_idx < n) match[cur_idx] = (int32_t)(i - soff);
                }
                if (BOXES && real) {
                    if (k == ECLIP) {
                        st_box(out, i, canon(cur_ctx));
                    } else {
                        defmask |= 1u << j;
                        def_L[j] = L;
                        def_own[j] = cur_own;
                        def_pos[j] = cur_pos;
                    }
                }
            }
            // every pop of a partition-incoming level leaves a record
            if (BOXES && cur_own < 0) {
                const int64_t ci = dP - L;
                if (ci >= 0 && ci < aP) {
                    int32_t sl = -1;
                    if (k == EBLEND && real && L >= 1 && cur_idx >= 0) {
                        int64_t R;
                        sl = (int32_t)incoming_slot(L, sm.runs, nruns, head, part, &R);
                    }
                    cr_slot[p0 + ci] = sl;
                    cr_c[p0 + ci] = (int32_t)i;
                }
            }
            --dep;
        }
    }
    if (!BOXES) return;

    // ---- unions that cross threads or partitions
    Box ttot = box_empty();
#pragma unroll
    for (int j = 0; j < K; ++j) ttot = unite(ttot, lout[j]);
    __syncthreads();  // the walk's reads of inc_ctx / jval / ucum are done
    uniontree_build(ut, ttot);
    {  // suffix unions after each of this thread's unmatched opens
        Box suf = box_empty();
#pragma unroll
        for (int p = K - 1; p >= 0; --p) {
            if ((wk.umask >> p) & 1u) sm.ucum[t * K + p] = suf;
            suf = unite(suf, lout[p]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (!((defmask >> j) & 1u)) continue;
        Box pre = box_empty();
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q < j) pre = unite(pre, lout[q]);
        const int64_t i = g0 + j;
        if (def_own[j] >= 0) {
            const int s = def_own[j];
            const Box u = unite(unite(sm.ucum[s * K + def_pos[j]], uniontree_range(ut, s + 1, t - 1)), pre);
            st_box(out, i, u);
            st_box(out, p0 + (int64_t)s * K + def_pos[j], u);
        } else {
            const int64_t ci = dP - def_L[j];
            if (ci >= 0 && ci < aP) st_box(cr_pre, p0 + ci, unite(uniontree_range(ut, 0, t - 1), pre));
        }
    }
    // surviving blend opens: union from the open to the end of the partition
    {
        const int sufmin = mintree_range_min(sm.mt, t + 1, W - 1);
        const int64_t baseP = (int64_t)myp.z;
        int jj = 0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            if (!((wk.umask >> p) & 1u)) continue;
            const int64_t L = (int64_t)base + 1 + jj;
            ++jj;
            if (L > (int64_t)sufmin || ks[p] != BBLEND) continue;
            const int64_t slot = L - baseP - 1;
            if (slot < 0 || slot >= T) continue;
            st_box(U_suf, p0 + slot, unite(sm.ucum[t * K + p], uniontree_range(ut, t + 1, W - 1)));
        }
    }
    if (t == 0) st_box(ptot, P, ut[1]);
}

// ------------------------------------------------ range unions over partitions
// Blocks of UB partitions: inclusive prefix and suffix unions inside each
// block, and block totals.
__global__ __launch_bounds__(UB) void k_ublocks(const float4 *__restrict__ ptot, int64_t M,
                                                float4 *__restrict__ upre, float4 *__restrict__ usuf,
                                                float4 *__restrict__ btot) {
    __shared__ Box sh[UB / WAVE];
    const int t = threadIdx.x;
    const int64_t B = blockIdx.x;
    const int64_t P = B * UB + t;
    const int64_t Pr = B * UB + (UB - 1 - t);
    const Box v = P < M ? ld_box(ptot, P) : box_empty();
    const Box vr = Pr < M ? ld_box(ptot, Pr) : box_empty();
    Box tot, tot2;
    const Box ex = block_excl_scan<UB / WAVE>(v, UniteOp{}, box_empty(), sh, &tot);
    const Box exr = block_excl_scan<UB / WAVE>(vr, UniteOp{}, box_empty(), sh, &tot2);
    if (P < M) st_box(upre, P, unite(ex, v));
    if (Pr < M) st_box(usuf, Pr, unite(exr, vr));
    if (t == 0) st_box(btot, B, tot);
}

// Sparse table over block totals: level l holds unions of 2^l blocks.
// Level 0 is the block totals themselves (the first nb entries of sp).
__global__ __launch_bounds__(1024) void k_usparse(float4 *__restrict__ sp, int64_t nb, int levels) {
    for (int l = 1; l < levels; ++l) {
        const int64_t half = (int64_t)1 << (l - 1);
        for (int64_t b = threadIdx.x; b < nb; b += 1024) {
            Box v = ld_box(sp, (l - 1) * nb + b);
            if (b + half < nb) v = unite(v, ld_box(sp, (l - 1) * nb + b + half));
            st_box(sp, l * nb + b, v);
        }
        __syncthreads();
    }
}

__device__ Box range_union(const float4 *ptot, const float4 *upre, const float4 *usuf,
                           const float4 *sp, int64_t nb, int64_t a, int64_t b) {
    Box u = box_empty();
    if (a > b) return u;
    const int64_t ba = a / UB, bb = b / UB;
    if (ba == bb) {
        for (int64_t q = a; q <= b; ++q) u = unite(u, ld_box(ptot, q));
        return u;
    }
    u = unite(ld_box(usuf, a), ld_box(upre, b));
    const int64_t l0 = ba + 1, l1 = bb - 1;
    if (l0 <= l1) {
        const int lv = 63 - __clzll((unsigned long long)(l1 - l0 + 1));
        u = unite(u, ld_box(sp, lv * nb + l0));
        u = unite(u, ld_box(sp, lv * nb + l1 - ((int64_t)1 << lv) + 1));
    }
    return u;
}

__global__ __launch_bounds__(W) void k_cross(const int4 *__restrict__ pinfo, int64_t M, int64_t n,
                                             const int32_t *__restrict__ U_idx,
                                             const float4 *__restrict__ U_suf,
                                             const int32_t *__restrict__ cr_slot,
                                             const int32_t *__restrict__ cr_c,
                                             const float4 *__restrict__ cr_pre,
                                             const float4 *__restrict__ ptot,
                                             const float4 *__restrict__ upre,
                                             const float4 *__restrict__ usuf,
                                             const float4 *__restrict__ sp, int64_t nb,
                                             float4 *__restrict__ out) {
    const int64_t Q = blockIdx.x;
    const int aQ = pinfo[Q].x;
    for (int ci = threadIdx.x; ci < aQ && ci < T; ci += W) {
        const int64_t slot = cr_slot[Q * T + ci];
        if (slot < 0 || slot >= Q * T) continue;
        const int64_t R = slot / T;
        const int64_t c = cr_c[Q * T + ci];
        const int64_t o = (int64_t)((uint32_t)U_idx[slot] & ~BLEND_BIT);
        if (o < 0 || o >= n || c < 0 || c >= n) continue;
        Box u = unite(ld_box(U_suf, slot), ld_box(cr_pre, Q * T + ci));
        u = unite(u, range_union(ptot, upre, usuf, sp, nb, R + 1, Q - 1));
        st_box(out, o, u);
        st_box(out, c, u);
    }
}

// ----------------------------------------------------------------- driver
hipEvent_t g_prof_before = nullptr, g_prof_after = nullptr;

static inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

FwdLayout fwd_layout(int64_t n, int64_t S) {
    FwdLayout L{};
    const int64_t M = n > 0 ? (n + T - 1) / T : 1;
    int64_t Mp = 1;
    while (Mp < M) Mp <<= 1;
    const int64_t nb = (M + UB - 1) / UB;
    int lv = 1;
    while (((int64_t)1 << lv) <= nb) ++lv;
    L.M = M;
    L.Mp = Mp;
    L.nb = nb;
    L.levels = lv;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    L.pinfo = take(sizeof(int4) * M);
    L.part = take(sizeof(int4) * M);
    L.mtree = take(sizeof(int) * 2 * Mp);
    L.jptr0 = take(sizeof(int32_t) * M);
    L.jptr1 = take(sizeof(int32_t) * M);
    L.jval0 = take(sizeof(float4) * M);
    L.jval1 = take(sizeof(float4) * M);
    L.U_idx = take(sizeof(int32_t) * M * T);
    L.U_cum = take(sizeof(float4) * M * T);
    L.U_suf = take(sizeof(float4) * M * T);
    L.cr_slot = take(sizeof(int32_t) * M * T);
    L.cr_c = take(sizeof(int32_t) * M * T);
    L.cr_pre = take(sizeof(float4) * M * T);
    L.runs = take(sizeof(int4) * M * RMAX);
    L.rhead = take(sizeof(int4) * M);
    L.ptot = take(sizeof(float4) * M);
    L.upre = take(sizeof(float4) * M);
    L.usuf = take(sizeof(float4) * M);
    L.sp = take(sizeof(float4) * nb * lv);
    L.status = take(sizeof(uint32_t) * (S > 0 ? S : 1));
    L.total = o;
    return L;
}

hipError_t fwd_run(bool boxes, const uint32_t *kind, const float4 *box, int64_t n,
                   const int64_t *off, int64_t S, int32_t *match, int32_t *pm, float4 *out,
                   void *ws, uint32_t *status, hipStream_t st) {
    const FwdLayout L = fwd_layout(n, off ? S : 1);
    char *w = (char *)ws;
    const int64_t nstat = off ? S : 1;
    if (!status) status = (uint32_t *)(w + L.status);
    k_zero_u32<<<(unsigned)((nstat + 255) / 256), 256, 0, st>>>(status, nstat);
    if (off) k_check_offsets<<<(unsigned)((S + 1 + 255) / 256), 256, 0, st>>>(off, S, n, status);
    if (n == 0) return hipGetLastError();
    const int64_t M = L.M;
    int4 *pinfo = (int4 *)(w + L.pinfo);
    int4 *part = (int4 *)(w + L.part);
    int *mtree = (int *)(w + L.mtree);
    int32_t *U_idx = (int32_t *)(w + L.U_idx);
    float4 *U_cum = (float4 *)(w + L.U_cum);
    if (boxes)
        k_reduce<true><<<(unsigned)M, W, 0, st>>>(kind, box, n, off, S, pinfo, U_idx, U_cum);
    else
        k_reduce<false><<<(unsigned)M, W, 0, st>>>(kind, box, n, off, S, pinfo, U_idx, U_cum);
    k_spine_scan<<<1, SPW, 0, st>>>(pinfo, M, part, mtree, L.Mp, off, S, n, status);
    int32_t *jp[2] = {(int32_t *)(w + L.jptr0), (int32_t *)(w + L.jptr1)};
    float4 *jv[2] = {(float4 *)(w + L.jval0), (float4 *)(w + L.jval1)};
    const unsigned gM = (unsigned)((M + 255) / 256);
    if (boxes)
        k_spine_link<true><<<gM, 256, 0, st>>>(pinfo, part, M, mtree, L.Mp, U_cum, jp[0], jv[0]);
    else
        k_spine_link<false><<<gM, 256, 0, st>>>(pinfo, part, M, mtree, L.Mp, U_cum, jp[0], jv[0]);
    int cur = 0;
    if (boxes) {
        int rounds = 0;
        while (((int64_t)1 << rounds) < M) ++rounds;
        for (int r = 0; r < rounds; ++r) {
            k_jump<<<gM, 256, 0, st>>>(jp[cur], jv[cur], jp[cur ^ 1], jv[cur ^ 1], M);
            cur ^= 1;
        }
    }
    float4 *U_suf = (float4 *)(w + L.U_suf);
    int32_t *cr_slot = (int32_t *)(w + L.cr_slot);
    int32_t *cr_c = (int32_t *)(w + L.cr_c);
    float4 *cr_pre = (float4 *)(w + L.cr_pre);
    float4 *ptot = (float4 *)(w + L.ptot);
    int4 *runs = (int4 *)(w + L.runs);
    int4 *rhead = (int4 *)(w + L.rhead);
    k_runs<<<gM, 256, 0, st>>>(pinfo, part, M, runs, rhead);
    const bool prof = g_prof_before && g_prof_after;
    if (prof) (void)hipEventRecord(g_prof_before, st);
    if (boxes)
        k_resolve<true><<<(unsigned)M, W, 0, st>>>(kind, box, n, off, S, pinfo, part, runs, rhead, jv[cur], U_idx,
                                                    U_cum, U_suf, cr_slot, cr_c, cr_pre, ptot, match,
                                                    pm, out, status);
    else
        k_resolve<false><<<(unsigned)M, W, 0, st>>>(kind, box, n, off, S, pinfo, part, runs, rhead, jv[cur],
                                                     U_idx, U_cum, U_suf, cr_slot, cr_c, cr_pre,
                                                     ptot, match, pm, out, status);
    if (prof) (void)hipEventRecord(g_prof_after, st);
    if (boxes) {
        float4 *upre = (float4 *)(w + L.upre);
        float4 *usuf = (float4 *)(w + L.usuf);
        float4 *sp = (float4 *)(w + L.sp);
        k_ublocks<<<(unsigned)L.nb, UB, 0, st>>>(ptot, M, upre, usuf, sp);
        k_usparse<<<1, 1024, 0, st>>>(sp, L.nb, L.levels);
        k_cross<<<(unsigned)M, W, 0, st>>>(pinfo, M, n, U_idx, U_suf, cr_slot, cr_c, cr_pre, ptot,
                                           upre, usuf, sp, L.nb, out);
    }
    return hipGetLastError();
}

}  // namespace tb
