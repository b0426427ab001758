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
//   k_spine_blocks / k_spine_top / k_spine_apply (/ k_spine_treetop)
//                 segmented depth scan over partitions; min tree of the
//                 partitions' lowest levels.  One launch of k_spine_apply
//                 when all partitions fit one block.
//   k_spine_link  owner link of each partition: the nearest earlier
//                 partition whose lowest level is smaller (it holds the
//                 stack entry just below); seeds pointer jumping.
//   k_jump        pointer jumping along owner links: the clip context at
//                 each partition's base level (the paper's pointer jumping,
//                 section "Parallel bounding boxes", Clips, applied to
//                 partitions instead of elements).
//   k_runs        the owner runs of each partition's incoming levels.
//                 k_link_small does the links, the jumping and the runs in
//                 one launch when the partitions fit one block.
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
//
// The same kernels serve the gradient pass (a (value, index) payload), the
// transform composition (an affine payload) and batched scenes (resets at
// scene starts).  The draw-object stream front end (k_cmp_count,
// k_cmp_scan, k_cmp_scatter, k_stream_match) extracts the tree's elements
// before the pipeline and translates the partners after it.
#include <mutex>
#include <type_traits>

#include "tb_common.h"
#include "tb_forward.h"

namespace tb {

// ------------------------------------------------------------------ utils
// clears the status words and the offsets flag word
__global__ void k_zero_status(uint32_t *status, int64_t cnt, uint32_t *flagw) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) status[i] = 0u;
    if (i == 0) *flagw = 0u;
}

// offsets must satisfy 0 = o[0] <= o[1] <= ... <= o[S] = n.  A violation
// anywhere makes every scene's status BAD_OFFSETS: the checking threads raise
// one flag word (zeroed with the status words), then k_offsets_flag copies
// it into all S words, so the cost stays O(S) however many offsets are bad.
__global__ void k_check_offsets(const int64_t *off, int64_t S, int64_t n, uint32_t *flagw) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S) return;
    bool bad = (s == 0 && off[0] != 0) || (s == S && off[S] != n) || (s < S && off[s] > off[s + 1]);
    if (bad) *flagw = 1u;  // every writer stores the same value
}

__global__ void k_offsets_flag(const uint32_t *flagw, int64_t S, uint32_t *status) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S && *flagw) status[s] |= ST_BAD_OFF;  // one thread per word: no atomics needed
}

// ---------------------------------------------------------------- k_reduce
// One workgroup of W threads per partition, K consecutive elements per
// thread (coalesced loads and stores).  The partition's bicyclic summary
// comes from DPP wave scans plus the wave totals (one barrier; one more when
// a scene starts in the partition), then the clip prefix of the surviving
// opens (one more) and the staging of the surviving opens (one more).
template <bool BOXES, class V, int KK, bool BRK = false, bool BAT = true>
__global__ __launch_bounds__(T / KK) void k_reduce(const uint32_t *__restrict__ kind,
                                              const float4 *__restrict__ box, int64_t n,
                                              const int64_t *__restrict__ off_in, int64_t S,
                                              int4 *__restrict__ pinfo,
                                              int32_t *__restrict__ U_idx, void *__restrict__ U_cum,
                                              const int64_t *__restrict__ n_dyn, uint32_t *__restrict__ zst) {
    constexpr int WW = T / KK, NW = WW / WAVE;  // threads and waves per partition
    // scene offsets (null for a single scene: a compile-time constant then)
    const int64_t *const off = BAT ? off_in : nullptr;
    __shared__ int4 sh_w[NW];  // per wave: scene start seen, depth sum, lowest depth
    __shared__ BicR sh_bic[NW];
    __shared__ V sh_b[NW];
    __shared__ int32_t sh_ui[T];
    __shared__ V sh_uc[BOXES ? T : 1];
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    const int wid = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: scalar loops over waves
    const int64_t P = blockIdx.x;
    const int64_t g0 = P * T + (int64_t)t * KK;
    // a single status word is cleared here rather than by a launch of its
    // own (every later writer of it runs after this kernel)
    if (zst && P == 0 && t == 0) *zst = 0u;
    if (n_dyn) {  // element count known on the device only: later partitions are empty
        n = *n_dyn;
        if (P * T >= n) {
            if (t == 0) pinfo[P] = make_int4(0, 0, 0, 0);
            return;
        }
    }

    uint32_t ks[KK];
    load_kinds<KK>(kind, n, g0, ks);
#pragma unroll
    for (int j = 0; j < KK; ++j)
        ks[j] = BRK ? bracket_kind(ks[j]) : ks[j] > 4u ? LEAF : Pay<V>::kAllOpens ? as_clip(ks[j]) : ks[j];
    const uint32_t rm = reset_mask<KK>(off, S, n, g0);
    const Walk wk = walk_kinds<KK>(ks, rm);
    const int b = (int)__popc(wk.umask);
    V bxs[KK];

    // Without a scene start in the partition (the common case) the summary
    // comes from plain integer scans: depth at each thread's start is the
    // sum of the earlier threads' net changes (b - a), cm = that depth - a
    // is the lowest depth the thread reaches, the partition pops -min cm of
    // the incoming stack, and a thread's unmatched opens (levels base+1 ..
    // base+b) survive unless a later thread reaches below them.  These are
    // DPP-fused adds and mins.  With a scene start the bicyclic products of
    // the threads (with resets) are scanned instead.
    constexpr int NONE = 1 << 24;  // above every depth a partition reaches
    const uint64_t rsb = __ballot(wk.rs);  // lanes of this wave with a scene start
    int wt, wmin;
    const int dl = wave_excl_scan(b - wk.a, AddOp{}, 0, &wt);
    const int cml = dl - wk.a;
    const int sufl = wave_excl_suffix_scan(cml, MinOp{}, NONE, &wmin);  // later lanes
    if (lane == 0) sh_w[wid] = make_int4(rsb != 0ull, wt, wmin, 0);
    __syncthreads();
    bool anyr = false;
#pragma unroll
    for (int w = 0; w < NW; ++w) anyr |= sh_w[w].x != 0;
    int base, ns, tota, totb, totr;
    if (!anyr) {  // block-uniform
        int offw = 0, acc = 0, minA = NONE, laterMin = NONE;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int4 x = sh_w[w];
            if (w == wid) offw = acc;
            minA = min(minA, acc + x.z);
            if (w > wid) laterMin = min(laterMin, acc + x.z);
            acc += x.y;
        }
        tota = minA < 0 ? -minA : 0;
        totb = acc + tota;
        totr = 0;
        base = offw + cml;
        const int mAfter = min(sufl == NONE ? NONE : sufl + offw, laterMin);
        ns = max(0, min(b, mAfter - base));
    } else {
        const BicR mine{wk.a, b, wk.rs ? 1 : 0};
        BicR wtot, wtot2;
        BicR pre = wave_excl_scan(mine, BicROp{}, BicR{0, 0, 0}, &wtot);
        BicR suf = wave_excl_suffix_scan(mine, BicROp{}, BicR{0, 0, 0}, &wtot2);
        if (lane == 0) sh_bic[wid] = wtot;
        __syncthreads();
        BicR before{0, 0, 0}, after{0, 0, 0}, tot{0, 0, 0};
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const BicR x = sh_bic[w];
            if (w < wid) before = bicr(before, x);
            tot = bicr(tot, x);
        }
#pragma unroll
        for (int w = NW - 1; w >= 0; --w)
            if (w > wid) after = bicr(sh_bic[w], after);
        pre = bicr(before, pre);
        suf = bicr(suf, after);
        const int D = pre.r ? pre.b : pre.b - pre.a;  // partition-relative unless a reset came first
        base = wk.rs ? 0 : D - wk.a;
        // later threads pop the last `suf.a` of this thread's unmatched opens
        ns = suf.r ? 0 : (b > suf.a ? b - suf.a : 0);
        tota = tot.a, totb = tot.b, totr = tot.r;
    }
    const int baseP = totr ? 0 : -tota;

    // clip prefix over the partition's surviving opens
    uint32_t surv = 0;  // positions of this thread's surviving unmatched opens
    {
        int jj = 0;
#pragma unroll
        for (int p = 0; p < KK; ++p) {
            if ((wk.umask >> p) & 1u) {
                if (jj < ns) surv |= 1u << p;
                ++jj;
            }
        }
    }
    V cum = Pay<V>::inf();
    if (BOXES) {
        // boxes of the clip opens that survive the partition
        uint32_t sc = 0;
#pragma unroll
        for (int p = 0; p < KK; ++p)
            if (((surv >> p) & 1u) && ks[p] == BCLIP) sc |= 1u << p;
#pragma unroll
        for (int p = 0; p < KK; ++p) bxs[p] = ((sc >> p) & 1u) ? Pay<V>::in(box, g0 + p) : Pay<V>::inf();
        // a wave without surviving clip opens has the identity for every
        // product (most waves of a partition that is not in a deep chain)
        V wagg = Pay<V>::inf();
        if (__ballot(sc != 0)) {
            V agg = Pay<V>::inf();
#pragma unroll
            for (int p = 0; p < KK; ++p)
                if ((sc >> p) & 1u) agg = isect(agg, bxs[p]);
            cum = wave_excl_scan(agg, IsectOp{}, Pay<V>::inf(), &wagg);
        }
        if (lane == 0) sh_b[wid] = wagg;
        __syncthreads();
        // earlier waves' products go in front, nearest wave first (the
        // combine need not be commutative); only waves with opens to stage
        if (__ballot(surv != 0)) {
#pragma unroll
            for (int w = NW - 2; w >= 0; --w)
                if (w < wid) cum = isect(sh_b[w], cum);
        }
    }

    // surviving opens fill slots [0, totb): staged in LDS, then written
    // with consecutive lanes on consecutive slots
    const int64_t slot0 = (int64_t)base - baseP;  // first surviving open's slot
    int jj = 0;
#pragma unroll
    for (int p = 0; p < KK; ++p) {
        if (!((surv >> p) & 1u)) continue;
        const int64_t slot = slot0 + jj;
        ++jj;
        if (slot < 0 || slot >= T) continue;
        sh_ui[slot] = (int32_t)((uint32_t)(g0 + p) | (ks[p] == BBLEND ? BLEND_BIT : 0u));
        if (BOXES) {
            cum = isect(cum, bxs[p]);  // the identity unless a clip
            sh_uc[slot] = cum;
        }
    }
    __syncthreads();
    const int nsv = totb < T ? totb : T;
    for (int sl = t; sl < nsv; sl += WW) {
        U_idx[P * T + sl] = sh_ui[sl];
        if (BOXES) Pay<V>::st(U_cum, P * T + sl, sh_uc[sl]);
    }
    if (t == 0) pinfo[P] = make_int4(tota, totb, totr, 0);
}

// ------------------------------------------------------------ spine kernels
// Segmented exclusive depth scan over the M partition summaries, in blocks
// of SB partitions (reduce, scan of block totals, apply), then partition
// records {d, cm, base, link} and a min tree over cm (each block builds its
// own subtree in LDS; one workgroup finishes the top).
constexpr int SB = 1024;

__device__ __forceinline__ Seg part_seg(int4 v) { return Seg{v.z, v.z ? v.y : v.y - v.x}; }

__global__ __launch_bounds__(SB) void k_spine_blocks(const int4 *__restrict__ pinfo, int64_t M,
                                                     int4 *__restrict__ bagg) {
    __shared__ Seg sh[SB / WAVE];
    __shared__ int shi[SB / WAVE];
    const int64_t P = (int64_t)blockIdx.x * SB + threadIdx.x;
    const int4 pv = P < M ? pinfo[P] : make_int4(0, 0, 0, 0);
    const Seg v = P < M ? part_seg(pv) : Seg{0, 0};
    Seg tot;
    block_excl_scan<SB / WAVE>(v, SegOp{}, Seg{0, 0}, sh, &tot);
    int atot;
    block_excl_scan<SB / WAVE>(pv.x, AddOp{}, 0, shi, &atot);
    if (threadIdx.x == 0) bagg[blockIdx.x] = make_int4(tot.r, tot.v, atot, 0);
}

// exclusive scan of the block totals (nbk <= SB * SPT), in place; checks
// that the whole sequence ends at depth 0
constexpr int SPT = 4;
__global__ __launch_bounds__(SB) void k_spine_top(int4 *__restrict__ bagg, int64_t nbk,
                                                  const int64_t *__restrict__ off, int64_t S,
                                                  int64_t n, uint32_t *__restrict__ status,
                                                  int *__restrict__ crtot) {
    __shared__ Seg sh[SB / WAVE];
    __shared__ int shi[SB / WAVE];
    const int t = threadIdx.x;
    Seg v[SPT], agg{0, 0};
    int av[SPT], aagg = 0;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int64_t b = (int64_t)t * SPT + q;
        const int4 x = b < nbk ? bagg[b] : make_int4(0, 0, 0, 0);
        v[q] = Seg{x.x, x.y};
        av[q] = x.z;
        agg = SegOp{}(agg, v[q]);
        aagg += x.z;
    }
    Seg tot;
    Seg ex = block_excl_scan<SB / WAVE>(agg, SegOp{}, Seg{0, 0}, sh, &tot);
    int atot;
    int aex = block_excl_scan<SB / WAVE>(aagg, AddOp{}, 0, shi, &atot);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
        const int64_t b = (int64_t)t * SPT + q;
        if (b < nbk) bagg[b] = make_int4(ex.r, ex.v, aex, 0);
        ex = SegOp{}(ex, v[q]);
        aex += av[q];
    }
    if (t == 0) {
        *crtot = atot;
        if (tot.v != 0 && n > 0) flag(status, off, S, n - 1, ST_UNBAL);
    }
}

// blocks cover [0, Mp): partition records, min-tree leaves and the block's
// subtree (padding leaves hold INT32_MAX).  With `single` (all partitions in
// one block) the block offsets are zero and this kernel also does the top
// kernel's work, so a small scene skips two launches.
__global__ __launch_bounds__(SB) void k_spine_apply(const int4 *__restrict__ pinfo, int64_t M,
                                                    const int4 *__restrict__ bex,
                                                    int4 *__restrict__ part, int *__restrict__ mtree,
                                                    int64_t Mp, int *__restrict__ crbase, bool single,
                                                    const int64_t *__restrict__ off, int64_t S,
                                                    int64_t n, uint32_t *__restrict__ status,
                                                    int *__restrict__ crtot) {
    __shared__ Seg sh[SB / WAVE];
    __shared__ int shi[SB / WAVE];
    __shared__ int lt[SB];
    const int t = threadIdx.x;
    const int64_t B = blockIdx.x;
    const int64_t P = B * SB + t;
    const int4 pv = P < M ? pinfo[P] : make_int4(0, 0, 0, 0);
    const Seg v = P < M ? part_seg(pv) : Seg{0, 0};
    Seg tot;
    const Seg loc = block_excl_scan<SB / WAVE>(v, SegOp{}, Seg{0, 0}, sh, &tot);
    int atot;
    const int aloc = block_excl_scan<SB / WAVE>(P < M ? pv.x : 0, AddOp{}, 0, shi, &atot);
    if (single && t == 0) {
        *crtot = atot;
        if (tot.v != 0 && n > 0) flag(status, off, S, n - 1, ST_UNBAL);
    }
    int cm = INT32_MAX;
    if (P < M) {
        const int4 bx = single ? make_int4(0, 0, 0, 0) : bex[B];
        crbase[P] = bx.z + aloc;
        const Seg ex = SegOp{}(Seg{bx.x, bx.y}, loc);
        const int d = ex.v;
        const int pre_m = d - pv.x;
        cm = pv.z ? SENT : pre_m;
        part[P] = make_int4(d, cm, pv.z ? 0 : pre_m, -1);
    }
    if (P < Mp) mtree[Mp + P] = cm;
    // subtree of this block: leaves lt[0..w), halving until one node
    const int64_t span = Mp < SB ? Mp : SB;
    lt[t] = cm;
    __syncthreads();
    int64_t base = Mp + B * SB;  // node index of this block's first leaf
    for (int64_t w = span / 2; w >= 1; w >>= 1) {
        base >>= 1;
        int m = INT32_MAX;
        if (t < w) m = min(lt[2 * t], lt[2 * t + 1]);
        __syncthreads();
        if (t < w) {
            lt[t] = m;
            mtree[base + t] = m;
        }
        __syncthreads();
    }
}

// levels above the block subtrees: nodes [1, Mp / SB)
__global__ __launch_bounds__(SB) void k_spine_treetop(int *__restrict__ mtree, int64_t Mp) {
    for (int64_t w = Mp / SB / 2; w >= 1; w >>= 1) {
        for (int64_t x = w + threadIdx.x; x < 2 * w; x += SB) mtree[x] = min(mtree[2 * x], mtree[2 * x + 1]);
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

// One partition's owner link (written to part[P].w) and, for payloads, the
// seed of pointer jumping: the context entry just below its base level.
template <bool BOXES, class V>
__device__ __forceinline__ void spine_link_one(int64_t P, const int4 *__restrict__ pinfo,
                                               int4 *__restrict__ part, const int *__restrict__ mtree,
                                               int64_t Mp, const void *__restrict__ U_cum,
                                               int32_t &ptr_out, V &val_out) {
    const int4 pr = part[P];
    const int64_t cm = pr.y;
    int64_t link = -1;
    if (cm != SENT) link = gtree_prev_less(mtree, Mp, P, cm);
    part[P].w = (int)link;
    V val = Pay<V>::inf();
    int64_t ptr = -1;
    if (BOXES && cm != SENT && cm > 0 && link >= 0) {
        const int64_t slot = cm - (int64_t)part[link].z - 1;
        if (slot >= 0 && slot < pinfo[link].y) {
            val = Pay<V>::ld(U_cum, link * T + slot);
            ptr = link;
        }
    }
    ptr_out = (int32_t)ptr;
    val_out = val;
}

template <bool BOXES, class V>
__global__ void k_spine_link(const int4 *__restrict__ pinfo, int4 *__restrict__ part, int64_t M,
                             const int *__restrict__ mtree, int64_t Mp,
                             const void *__restrict__ U_cum, int32_t *__restrict__ jptr,
                             void *__restrict__ jval) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M) return;
    int32_t ptr;
    V val;
    spine_link_one<BOXES, V>(P, pinfo, part, mtree, Mp, U_cum, ptr, val);
    if (!BOXES) return;
    jptr[P] = ptr;
    Pay<V>::st(jval, P, val);
}

// owners a pointer-jumping round covers per input pointer (JH^r after r rounds)
constexpr int JH = 8;

template <class V>
__global__ void k_jump(const int32_t *__restrict__ ptr_in, const void *__restrict__ val_in,
                       int32_t *__restrict__ ptr_out, void *__restrict__ val_out, int64_t M) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= M) return;
    // JH - 1 hops per round, so fewer launches: each hop puts the next
    // owner's value in front (ancestor-first order).
    int32_t p = ptr_in[P];
    V v = Pay<V>::ld(val_in, P);
#pragma unroll
    for (int h = 1; h < JH; ++h) {
        if (p >= 0) {
            v = isect(Pay<V>::ld(val_in, p), v);
            p = ptr_in[p];
        }
    }
    ptr_out[P] = p;
    Pay<V>::st(val_out, P, v);
}

constexpr int JS = 1024;  // partitions handled by one workgroup in k_link_small

// ---------------------------------------------------------------- k_runs
// Owner runs of each partition's incoming levels [max(preM,1), dP]: walking
// the owner links from P-1, each owner R holds a contiguous range of levels
// (its surviving opens).  One thread per partition; many chains are walked
// at once, which hides the dependent loads.  Up to RMAX runs are stored;
// head = {count, next owner, next top level, complete}.
__device__ __forceinline__ void runs_one(int64_t P, const int4 *__restrict__ pinfo,
                                         const int4 *__restrict__ part, int4 *__restrict__ runs,
                                         int4 *__restrict__ rhead) {
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

__global__ void k_runs(const int4 *__restrict__ pinfo, const int4 *__restrict__ part, int64_t M,
                       int4 *__restrict__ runs, int4 *__restrict__ rhead) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P < M) runs_one(P, pinfo, part, runs, rhead);
}

// Links, pointer jumping and owner runs in one launch when the partitions
// fit one block (M <= JS): the links are published to the block by a
// barrier, and the jumping rounds run in LDS.
template <bool BOXES, class V>
__global__ __launch_bounds__(JS) void k_link_small(const int4 *__restrict__ pinfo,
                                                   int4 *__restrict__ part, int64_t M,
                                                   const int *__restrict__ mtree, int64_t Mp,
                                                   const void *__restrict__ U_cum,
                                                   int32_t *__restrict__ jptr, void *__restrict__ jval,
                                                   int rounds, int4 *__restrict__ runs,
                                                   int4 *__restrict__ rhead) {
    __shared__ int32_t sp[JS];
    __shared__ V sv[BOXES ? JS : 1];
    const int P = threadIdx.x;
    int32_t p = -1;
    V v = Pay<V>::inf();
    if (P < M) spine_link_one<BOXES, V>(P, pinfo, part, mtree, Mp, U_cum, p, v);
    __syncthreads();  // every link is in part[].w
    if (BOXES) {
        for (int r = 0; r < rounds; ++r) {
            sp[P] = p;
            sv[P] = v;
            __syncthreads();
            if (p >= 0) {
                v = isect(sv[p], v);  // ancestor first
                p = sp[p];
            }
            __syncthreads();
        }
        if (P < M) {
            jptr[P] = p;
            Pay<V>::st(jval, P, v);
        }
    }
    if (P < M) runs_one(P, pinfo, part, runs, rhead);
}

// ------------------------------------------------------------- k_resolve

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
                                 const int4 *__restrict__ part, int64_t M, int64_t *owner) {
    int64_t R = -1, base = 0;
    const int r = find_run(runs, nruns, L);
    if (r >= 0) {
        R = runs[r].x;
        base = runs[r].w;
    } else if (!head.w) {
        int64_t RR = head.y, hi = head.z;
        while (RR >= 0 && RR < M && hi >= L) {
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
    if (R < 0 || R >= M || L - base - 1 < 0 || L - base - 1 >= T) return -1;
    return R * T + (L - base - 1);
}

template <bool BOXES, class V, int KK>
struct ResolveSmem {
    static constexpr int WW = T / KK, NW = WW / WAVE;
    struct EarlyTables {
        V jval[BOXES ? WW : 1];
        // the contexts after jumping (small payloads: their own array
        // saves a barrier; larger ones overwrite jval, to keep LDS low)
        V jfin[BOXES && sizeof(V) <= 24 ? WW : 1];
        int inc_idx[T + 1];
        // per thread: {lowest level (SENT after a scene start), owner
        // thread or -1, base level, first cx entry | unmatched-open mask
        // << 16 | mask of those that are clips << (16 + KK)}; one LDS
        // read per owner-chain hop
        int4 tinfo[WW];
        int mt[2 * WW];
        int jptr[WW];
    };
    // per wave, the in-partition cross-thread blend closes gathered into the
    // space the early tables leave beside the union tree
    static constexpr int UTB = (BOXES ? 2 * WW : 1) * (int)sizeof(V);
    static constexpr int DCAP_RAW = ((int)sizeof(EarlyTables) - UTB) / (NW * (8 + (int)sizeof(V)));
    static constexpr int DCAP = DCAP_RAW > 0 ? DCAP_RAW : 1;
    int4 runs[RMAX];
    // Until the walk ends: the clip context at each thread's base level, the
    // incoming levels [preM, dP] (entry x = level preM + x: the open's
    // index | BLEND_BIT, or -1 for the root), the per-thread lookup records,
    // the min tree and the jumping pointers.  Afterwards: the union tree
    // over threads, which overlays them all.
    union Early {
        EarlyTables w;
        V ut[BOXES ? 2 * WW : 1];
        struct {
            V ut_space[BOXES ? 2 * WW : 1];
            int2 item[NW * DCAP];
            V pre[NW * DCAP];
        } d;
    } e;
    static_assert(KK <= 8 && T < 0xFFFF, "tinfo packs two KK-bit masks above a 16-bit entry");
    // Clip contexts.  Entries [0, aP] belong to the incoming levels; from
    // aP + 1 on come the unmatched opens of each thread in order (thread t's
    // from aP + 1 + tub[t]) with their local clip prefix, which the union
    // phase replaces by suffix unions.  A partition's incoming pops (aP) and
    // its threads' unmatched opens are different elements, so T + 1 entries
    // always suffice.
    V cx[BOXES ? T + 1 : 1];
    SegU sh_seg[NW];
    V wtot[NW];  // union of each wave's leaves
};

template <bool BOXES, class V, class SINK, int KK, bool BRK = false, bool BAT = true>
__global__ __launch_bounds__(T / KK) __attribute__((amdgpu_waves_per_eu(3))) void k_resolve(
    const uint32_t *__restrict__ kind, const float4 *__restrict__ box, int64_t n,
    const int64_t *__restrict__ off_in, int64_t S, const int4 *__restrict__ pinfo,
    const int4 *__restrict__ part, const int4 *__restrict__ runs_g,
    const int4 *__restrict__ rhead_g, const void *__restrict__ base_ctx,
    const int32_t *__restrict__ U_idx, const void *__restrict__ U_cum,
    void *__restrict__ U_suf, const int *__restrict__ crbase, int32_t *__restrict__ cr_slot,
    int32_t *__restrict__ cr_c, void *__restrict__ cr_pre, void *__restrict__ ptot,
    int32_t *__restrict__ match, int32_t *__restrict__ pm, SINK sink,
    uint32_t *__restrict__ status, const int64_t *__restrict__ n_dyn) {
    constexpr int WW = T / KK, NW = WW / WAVE;  // threads and waves per partition
    // scene offsets (null for a single scene: a compile-time constant then)
    const int64_t *const off = BAT ? off_in : nullptr;
    __shared__ ResolveSmem<BOXES, V, KK> sm;
    V *ut = sm.e.ut;  // valid once the walk is over
    const int t = threadIdx.x, lane = t & (WAVE - 1), wbase = t & ~(WAVE - 1);
    const int wid = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform: scalar loops over waves
    // Element indices and levels fit in 32 bits (n < 2^31); element indices
    // are unsigned so that a last partition past 2^31 - T cannot overflow.
    const uint32_t P = blockIdx.x;
    const uint32_t M = gridDim.x;
    const uint32_t p0 = P * T;
    const uint32_t g0 = p0 + (uint32_t)t * KK;
    if (n_dyn) {  // element count known on the device only
        n = *n_dyn;
        if ((int64_t)p0 >= n) {  // an empty partition: its leaf union is EMPTY
            if (BOXES && Pay<V>::kUnions && t == 0) Pay<V>::st(ptot, P, Pay<V>::empty());
            return;
        }
    }
    const uint32_t un = (uint32_t)n;
    const int4 myp = part[P];
    const int dP = myp.x;
    const int aP = pinfo[P].x;
    const int preM = dP - aP;  // lowest incoming level any element here can see
    const int4 head = rhead_g[P];
    const int nruns = head.x;
    const int rbase = crbase[P];  // this partition's close records start here

    // ---- loads: inputs, owner runs
    uint32_t kr[KK], ks[KK];
    load_kinds<KK>(kind, n, g0, kr);
    V bx[KK];
    if (BOXES) {
#pragma unroll
        for (int j = 0; j < KK; ++j) bx[j] = (g0 + j < n) ? Pay<V>::in(box, g0 + j) : Pay<V>::empty();
    }
    uint32_t spos[SINK::kPos ? KK : 1];  // output positions of this thread's rows
    if constexpr (SINK::kPos) {
#pragma unroll
        for (int j = 0; j < KK; ++j) spos[j] = (g0 + j < n) ? sink.pos(g0 + j) : ~0u;
    }
    if (t < RMAX) sm.runs[t] = runs_g[P * RMAX + t];
#pragma unroll
    for (int j = 0; j < KK; ++j)
        ks[j] = BRK ? bracket_kind(kr[j]) : kr[j] > 4u ? LEAF : Pay<V>::kAllOpens ? as_clip(kr[j]) : kr[j];
    static_assert(!BRK || !BOXES, "typed brackets are matched without payloads");
    const uint32_t rm = reset_mask<KK>(off, S, n, g0);
    __syncthreads();

    // ---- gather the incoming levels [preM, dP] (issued now, stored later)
    constexpr int NG = (T + WW) / WW;  // entries per thread
    int g_idx[NG];
    V g_ctx[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        g_idx[q] = -1;
        g_ctx[q] = Pay<V>::inf();
        const int x = t + q * WW;
        const int L = preM + x;
        if (x > aP) continue;
        int64_t R = -1, slot = -1;
        if (L >= 1) slot = incoming_slot(L, sm.runs, nruns, head, part, M, &R);
        // if level L is popped here, that pop is close record aP - x
        if (BOXES && x >= 1 && (uint32_t)(rbase + aP - x) < un) cr_slot[rbase + aP - x] = (int32_t)slot;
        if (slot < 0) continue;
        g_idx[q] = U_idx[slot];
        if (BOXES) g_ctx[q] = isect(Pay<V>::ld(base_ctx, R), Pay<V>::ld(U_cum, slot));
    }

    // ---- per-thread walk and thread-level depths
    const Walk wk = walk_kinds<KK>(ks, rm);
    const int b = __popc(wk.umask);
    SegU segtot;
    const SegU ex = block_excl_scan<NW, SegU, SegUOp, false>(SegU{wk.rs ? 1 : 0, wk.rs ? b : b - wk.a, b},
                                                             SegUOp{}, SegU{0, 0, 0}, sm.sh_seg, &segtot);
    const int ub = aP + 1 + ex.u;  // this thread's first entry in cx
    const int Dt = ex.r ? ex.v : dP + ex.v;  // absolute depth at thread start
    const int pre_m = Dt - wk.a;
    const int cm = wk.rs ? SENT : (int)pre_m;
    const int base = wk.rs ? 0 : (int)pre_m;
    {
        uint32_t clipm = 0;
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if (ks[j] == BCLIP) clipm |= 1u << j;
        sm.e.w.tinfo[t] = make_int4(cm, -1, base, (int)((uint32_t)ub | (wk.umask << 16) | ((clipm & wk.umask) << (16 + KK))));
    }
    {  // this thread's unmatched opens: element index (| BLEND_BIT) and clip prefix
        V c = Pay<V>::inf();
        int e = ub;
#pragma unroll
        for (int p = 0; p < KK; ++p) {
            if ((wk.umask >> p) & 1u) {
                if (BOXES && ks[p] == BCLIP) c = isect(c, bx[p]);
                if (e <= T) {
                    sm.e.w.inc_idx[e] = (int)((g0 + p) | (ks[p] == BBLEND ? BLEND_BIT : 0u));
                    if (BOXES) sm.cx[e] = c;
                }
                ++e;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const int x = t + q * WW;
        if (x > aP) continue;
        sm.e.w.inc_idx[x] = g_idx[q];
        if (BOXES) sm.cx[x] = g_ctx[q];
        // a clip level popped here: its close record carries the open's full
        // context, which is the pair's box (blend records get their prefix
        // union in the union phase)
        if (BOXES && x >= 1 && g_idx[q] != -1 && !((uint32_t)g_idx[q] & BLEND_BIT) &&
            (uint32_t)(rbase + aP - x) < un)
            Pay<V>::st(cr_pre, rbase + aP - x, g_ctx[q]);
    }
    int wmin0;
    int premin = wave_excl_scan(cm, MinOp{}, INT32_MAX, &wmin0);  // lowest level of earlier lanes
    mintree_build<WW>(sm.e.w.mt, cm);  // its barrier also publishes everything above

    // levels at or below `lowtop` are held by no earlier thread of this
    // partition: they come from earlier partitions (the LDS table).
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
        if (w < wid) premin = min(premin, sm.e.w.mt[NW + w]);  // wave nodes of the min tree
    const int lowtop = min(premin, Dt);
    // lowest level any later thread reaches: an unmatched open of this thread
    // at a level not above it survives the partition
    int wmin1;
    int sufmin = wave_excl_suffix_scan(cm, MinOp{}, INT32_MAX, &wmin1);
#pragma unroll
    for (int w = 1; w < NW; ++w)
        if (w > wid) sufmin = min(sufmin, sm.e.w.mt[NW + w]);
    // owner links between threads: the entry just below a thread's lowest
    // level belongs to the nearest earlier thread with a smaller lowest level
    const int tl = wk.rs ? -1 : mintree_prev_less<WW>(sm.e.w.mt, t, cm);
    sm.e.w.tinfo[t].y = tl;

    // ---- clip context at each thread's base level: pointer jumping along
    // owner threads, first inside the wave with shuffles, then across waves.
    if (BOXES) {
        V v = Pay<V>::inf();
        int ptr = -1;
        if (!wk.rs && pre_m > 0) {
            const int s = tl;
            if (s >= 0) {
                const int4 ti = sm.e.w.tinfo[s];
                const int jj = pre_m - ti.z - 1;
                const uint32_t um = ((uint32_t)ti.w >> 16) & ((1u << KK) - 1u);
                const int e = (ti.w & 0xFFFF) + (int)jj;
                if (jj >= 0 && jj < __popc(um) && e <= T) {
                    v = sm.cx[e];
                    ptr = s;
                }
            } else {
                const int x = pre_m - preM;
                if (x >= 0 && x <= aP) v = sm.cx[x];
            }
        }
        for (int r = 0; r < 6 && __ballot(ptr >= wbase); ++r) {  // until no lane points inside the wave
            const bool in = ptr >= wbase;
            const int src = in ? ptr - wbase : lane;
            const V vv = shfl_idx(v, src);
            const int pp = __shfl(ptr, src, WAVE);
            if (in) {
                v = isect(vv, v);  // the owner's context comes first
                ptr = pp;
            }
        }
        // Across waves every pointer now leaves its wave, so a chain has at
        // most NW - 1 more hops: follow it through the published values
        // (each hop's value is fixed, so hops compose, owner first).
        sm.e.w.jval[t] = v;
        sm.e.w.jptr[t] = ptr;
        __syncthreads();  // also publishes tlink
#pragma unroll
        for (int h = 0; h < NW - 1; ++h) {
            if (ptr >= 0) {
                v = isect(sm.e.w.jval[ptr], v);
                ptr = sm.e.w.jptr[ptr];
            }
        }
        if (sizeof(V) <= 24) {
            sm.e.w.jfin[t] = v;
        } else {
            __syncthreads();  // every read of the published values is done
            sm.e.w.jval[t] = v;
        }
        __syncthreads();
    } else {
        __syncthreads();  // publishes tlink
    }

    // ---- this thread's elements in order.  The thread's own opens form a
    // stack held as a bit mask of positions (top = highest bit), each with
    // the clip context inside it; levels below come from lookups.  Rows are
    // collected in registers and written once at the end.
    int64_t sid = off ? scene_of(off, S, g0) : 0;
    int soff = off ? (int)off[sid] : 0;
    const int soff0 = soff;  // the thread's first scene
    uint32_t mask = 0;    // open positions on the local stack
    uint32_t clipm = 0;   // positions holding BEGIN_CLIP
    uint32_t leafm = 0;   // positions holding leaves (the only rows unions read)
    uint32_t keep = 0;    // rows this thread writes at the end
    uint32_t mkeep = 0;   // match rows this thread writes at the end
    uint32_t lbm = 0;     // closes of blends opened in this thread
    uint32_t rchk = 0;    // typed brackets: closes whose open's token is checked after the walk
    uint32_t defmask = 0; // closes of blends opened before this thread
    uint32_t rmm = 0;     // closes whose open lies in an earlier thread of this partition
    uint32_t recm = 0;    // closes that leave a close record
    int crci[KK];         // close record index within this partition
    using ErrT = std::conditional_t<(KK + 1) * 4 <= 32, uint32_t, uint64_t>;
    ErrT errs = 0;        // status bits, 4 per element; element g0 - 1 at bit 4KK
    bool rseen = false;
    int dep = Dt;
    V octx[KK], res[KK];
    int mv[KK];
    uint32_t lbp = 0;  // 3 bits per position: the local open a blend close matches
    // per deferred blend close, packed: owner thread + 1 (0 = an earlier
    // partition), its position and cx entry; or, for an earlier partition,
    // the close record's index within this partition
    uint32_t dfw[KK];
    // the stack entry at level `cur_L` seen from this thread's start; the
    // levels asked for only decrease, so the owner search moves left along
    // owner links from the previous thread
    int cur_L = INT32_MIN, cur_idx = -1;
    int own_s = t - 1;
    int cur_kind = -1, cur_own = -1, cur_pos = -1, cur_ent = -1;
    V cur_ctx = Pay<V>::inf();
#pragma unroll
    for (int j = 0; j < KK; ++j) {
        octx[j] = Pay<V>::inf();
        res[j] = Pay<V>::empty();
        mv[j] = -1;
        dfw[j] = 0;
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < KK; ++j) {
        const uint32_t i = g0 + j;
        const bool real = i < un;
        const uint32_t bit = 1u << j;
        if ((rm >> j) & 1u) {
            if (real && i > 0 && dep != 0) errs |= (ErrT)ST_UNBAL << (j > 0 ? 4 * (j - 1) : 4 * KK);  // element i - 1
            mask = 0;
            rseen = true;
            dep = 0;
            if (off && real) {
                sid = scene_of(off, S, i);
                soff = (int)off[sid];
            }
        }
        if (!BRK && real && kr[j] > 4u) errs |= (ErrT)ST_BAD_KIND << (4 * j);
        const int tp = mask ? msb32(mask) : -1;
        if (tp < 0 && !rseen && cur_L != dep) {
            // straight-line lookup: the holder thread (levels above lowtop)
            // or the incoming table; both name an entry of inc_idx and cx
            cur_L = dep;
            const bool tabp = dep <= lowtop;
            int4 ti = make_int4(0, -1, 0, 0);
            if (!tabp) {
                // each hop reads a record's lowest level and owner link in
                // one 8-byte LDS read; the rest of the record after the walk
                const int2 *txy = reinterpret_cast<const int2 *>(sm.e.w.tinfo);
                int2 xy = txy[2 * (own_s >= 0 ? own_s : 0)];
                while (own_s >= 0 && xy.x >= dep) {
                    own_s = xy.y;
                    xy = txy[2 * (own_s >= 0 ? own_s : 0)];
                }
                const int2 zw = txy[2 * (own_s >= 0 ? own_s : 0) + 1];
                ti = make_int4(xy.x, xy.y, zw.x, zw.y);
            }
            const int s = tabp ? -1 : own_s;
            const int jj = dep - ti.z - 1;
            const uint32_t um = ((uint32_t)ti.w >> 16) & ((1u << KK) - 1u);
            const int eo = (ti.w & 0xFFFF) + jj;
            const bool okown = s >= 0 && jj >= 0 && jj < (int)__popc(um) && eo <= T;
            const int x = dep - preM;
            const bool oktab = tabp && dep >= 1 && x >= 0 && x <= aP;
            const int ent = oktab ? x : okown ? eo : 0;
            const int u = sm.e.w.inc_idx[ent];
            const V c = BOXES ? sm.cx[ent] : Pay<V>::inf();
            const V jv = !BOXES ? Pay<V>::inf() : sizeof(V) <= 24 ? sm.e.w.jfin[okown ? s : 0] : sm.e.w.jval[okown ? s : 0];
            const bool hit = (oktab || okown) && u != -1;
            cur_idx = hit ? (int)((uint32_t)u & ~BLEND_BIT) : -1;
            cur_kind = !hit ? -1 : ((uint32_t)u & BLEND_BIT) ? (int)BBLEND : (int)BCLIP;
            if (BOXES) cur_ctx = vsel(hit, vsel(okown, isect(jv, c), c), Pay<V>::inf());
            cur_own = hit && okown ? s : -1;
            cur_pos = cur_idx - (int)(p0 + (uint32_t)s * KK);
            cur_ent = eo;
        }
        // the top of the stack before this element: a local open, the scene
        // root after a reset, or the looked-up entry
        int top = tp >= 0 ? (int)(g0 + tp) : rseen ? -1 : cur_idx;
        V ctx = vsel(rseen, Pay<V>::inf(), cur_ctx);
        if (BOXES && j > 0) {
            uint32_t tpm = tp >= 0 ? 1u << tp : 0u;
            asm("" : "+v"(tpm));  // opaque: selects, not an indexed load
#pragma unroll
            for (int q = 0; q < j; ++q) ctx = vsel(((tpm >> q) & 1u) != 0, octx[q], ctx);
        }
        if (pm && real) pm[i] = top >= 0 ? (int32_t)(top - soff) : -1;
        // every case below is computed with selects: the wave runs one
        // straight-line step per element however its lanes' kinds differ
        const uint32_t k = ks[j];
        const bool isleaf = k == LEAF;
        const bool isopen = is_open(k);
        const bool isclose = !isleaf && !isopen;
        const bool lclose = isclose && tp >= 0;            // closes an open of this thread
        const bool rootclose = isclose && tp < 0 && rseen;  // closes below its scene's root
        const bool rclose = isclose && tp < 0 && !rseen;    // closes a level held before this thread
        const bool rok = rclose && dep > 0 && cur_idx >= 0;
        // pops of levels held by earlier partitions leave a close record, and
        // the cross-partition kernel writes both rows and both match entries
        const int ci = dP - dep;
        const bool rec = BOXES && rclose && cur_own < 0 && ci >= 0 && ci < aP && (uint32_t)(rbase + ci) < un;
        // so does a clip open that survives this partition
        const bool sclip = BOXES && k == BCLIP && ((wk.umask >> j) & 1u) && dep + 1 <= sufmin;
        const int tps = tp < 0 ? 0 : tp;
        const uint32_t pbit = lclose ? (1u << tps) : 0u;
        if (BOXES) {
            const V ix = isect(ctx, bx[j]);
            octx[j] = vsel(k == BCLIP, ix, ctx);
            // leaf: its clipped box; BEGIN_CLIP: likewise; END_CLIP: the
            // context inside its open.  Blend rows are filled in later.
            res[j] = canon(vsel((isleaf && Pay<V>::kLeafOwn) || k == BCLIP, ix, ctx));
        }
        bool mism;
        if (BRK) {
            // a close must carry its open's token plus one; an open in an
            // earlier thread is checked after the walk (a global read)
            uint32_t otok = 0;
#pragma unroll
            for (int q = 0; q < j; ++q)
                if (q == tps) otok = kr[q];
            mism = lclose && kr[j] != otok + 1u;
            rchk |= (rok && real) ? bit : 0u;
        } else {
            mism = (lclose && ((k == ECLIP) != (((clipm >> tps) & 1u) != 0))) ||
                   (rok && ((k == ECLIP) != (cur_kind == (int)BCLIP)));
        }
        errs |= (real && mism) ? (ErrT)ST_MISMATCH << (4 * j) : 0u;
        errs |= (real && (rootclose || (rclose && !rok))) ? (ErrT)ST_UNBAL << (4 * j) : 0u;
        leafm |= isleaf ? bit : 0u;
        clipm |= k == BCLIP ? bit : 0u;
        keep |= (isleaf || (k == BCLIP && !sclip) || (k == ECLIP && (lclose || (rok && !rec)))) ? bit : 0u;
        keep |= (lclose && k == EBLEND) ? (bit | pbit) : 0u;
        lbm |= (lclose && k == EBLEND) ? bit : 0u;
        lbp |= (uint32_t)tps << (3 * j);
        mkeep |= (isleaf || lclose || (rok && !rec)) ? bit : 0u;
        mkeep |= pbit;
        mv[j] = lclose ? (int32_t)(g0 + tps - soff) : rok ? (int32_t)(cur_idx - soff) : -1;
#pragma unroll
        for (int q = 0; q < j; ++q)
            if (lclose && q == tp) mv[q] = (int32_t)(i - soff);
        // the open's match entry, written after the walk
        rmm |= (rok && !rec && real && (uint32_t)cur_idx < un) ? bit : 0u;
        const bool dfb = BOXES && rok && k == EBLEND && real;
        defmask |= dfb ? bit : 0u;
        dfw[j] = !dfb ? 0u
                      : cur_own >= 0 ? (uint32_t)(cur_own + 1) | ((uint32_t)cur_pos << 9) | ((uint32_t)cur_ent << 12)
                                     : (uint32_t)(dP - dep) << 12;
        // close records, written after the walk
        recm |= rec ? bit : 0u;
        crci[j] = ci;
        mask = isopen ? (mask | bit) : (mask & ~pbit);
        dep += isopen ? 1 : (lclose || rclose) ? -1 : 0;
    }
    // pops of levels held by earlier threads or partitions happen before any
    // scene start of this thread, so they share the thread's first scene
    if (match && rmm) {
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if ((rmm >> j) & 1u) match[mv[j] + soff0] = (int32_t)(g0 + j - soff0);
    }
    if (BOXES && recm) {
        // the close's position, with the top bit set for a blend; the slot
        // was written by the gather
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if ((recm >> j) & 1u) cr_c[rbase + crci[j]] = (int32_t)((g0 + j) | (ks[j] == EBLEND ? 0x80000000u : 0u));
    }
    if (BRK && __ballot(rchk != 0)) {
        // closes of opens held by earlier threads: compare with the open's
        // token, every read in flight before the first compare
        uint32_t otok[KK];
#pragma unroll
        for (int j = 0; j < KK; ++j) {
            const uint32_t oi = (uint32_t)mv[j] + (uint32_t)soff;
            otok[j] = ((rchk >> j) & 1u) && oi < un ? kind[oi] : 0u;
        }
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if (((rchk >> j) & 1u) && kr[j] != otok[j] + 1u) errs |= (ErrT)ST_MISMATCH << (4 * j);
    }
    if (errs) {  // malformed input only: raise each element's bits in its scene's word
#pragma unroll
        for (int j = 0; j <= KK; ++j) {
            const uint32_t bj = (uint32_t)(errs >> (4 * j)) & 0xFu;
            if (bj) flag(status, off, S, j < KK ? (int64_t)g0 + j : (int64_t)g0 - 1, bj);
        }
    }
    // Leaf rows (EMPTY elsewhere) and their prefix unions pu[j] (leaves
    // before position j), all with selects: every lane runs the same steps.
    V pu[KK + 1], sa[KK];  // sa[p]: union of the leaves after position p
    if (BOXES) {
        V lr[KK];
#pragma unroll
        for (int j = 0; j < KK; ++j) lr[j] = vsel(((leafm >> j) & 1u) != 0, res[j], Pay<V>::empty());
        pu[0] = Pay<V>::empty();
#pragma unroll
        for (int j = 0; j < KK; ++j) pu[j + 1] = unite(pu[j], lr[j]);
        sa[KK - 1] = Pay<V>::empty();
#pragma unroll
        for (int j = KK - 2; j >= 0; --j) sa[j] = unite(sa[j + 1], lr[j + 1]);
        // blends opened and closed in this thread: the union of the leaves
        // strictly between open p and close j
#pragma unroll
        for (int j = 1; j < KK; ++j) {
            const bool lb = (lbm >> j) & 1u;
            const int p = (lbp >> (3 * j)) & 7u;
            V acc = Pay<V>::empty(), u = Pay<V>::empty();
#pragma unroll
            for (int q = j - 1; q >= 0; --q) {
                u = vsel(q == p, acc, u);
                acc = unite(acc, lr[q]);
            }
            res[j] = vsel(lb, u, res[j]);
            // the open's row too; an opaque one-hot mask keeps the compiler
            // from turning the selects into an indexed (scratch) store
            uint32_t pm1 = lb ? 1u << p : 0u;
            asm("" : "+v"(pm1));  // opaque to the compiler
#pragma unroll
            for (int q = 0; q < j; ++q) res[q] = vsel(((pm1 >> q) & 1u) != 0, u, res[q]);
        }
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if (((keep >> j) & 1u) && g0 + j < un) {
                if constexpr (SINK::kPos)
                    sink.emit_at(spos[j], res[j]);
                else
                    sink.emit(g0 + j, res[j]);
            }
    }
    if (match) {
#pragma unroll
        for (int j = 0; j < KK; ++j)
            if (((mkeep >> j) & 1u) && g0 + j < un) match[g0 + j] = mv[j];
    }
    if (!BOXES || !Pay<V>::kUnions) return;

    // ---- unions that cross threads or partitions.  Prefix and suffix
    // unions over threads come from wave scans plus the wave totals; only
    // blends opened and closed in different threads of this partition need
    // an arbitrary range, answered from a union tree over threads.
    const V ttot = pu[KK];
    V wsuf_dummy;
    const V wsuf = wave_excl_suffix_scan(ttot, UniteOp{}, Pay<V>::empty(), &wsuf_dummy);
    __syncthreads();  // the walk's reads of the early tables and cx are done
    V wtot_u;
    const V wpre = uniontree_scan<V, WW>(ut, ttot, &wtot_u);
    if (lane == 0) sm.wtot[wid] = wtot_u;
    // suffix unions after each of this thread's unmatched opens
#pragma unroll
    for (int p = 0; p < KK; ++p) {
        const int e = ub + (int)__popc(wk.umask & ((1u << p) - 1u));
        if (((wk.umask >> p) & 1u) && e <= T) sm.cx[e] = sa[p];
    }
    __syncthreads();
    V pre_t = wpre, suf_t = wsuf, all = Pay<V>::empty();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const V x = sm.wtot[w];
        if (w < wid) pre_t = unite(pre_t, x);
        if (w > wid) suf_t = unite(suf_t, x);
        all = unite(all, x);
    }
    // closes of blends opened in an earlier partition: the prefix part
    uint32_t dloc = 0;  // closes of blends opened in an earlier thread of this partition
#pragma unroll
    for (int j = 0; j < KK; ++j) {
        if (!((defmask >> j) & 1u)) continue;
        if (dfw[j] & 0x1FFu) {  // owner thread in this partition
            dloc |= 1u << j;
            continue;
        }
        const int ci = (int)(dfw[j] >> 12);
        if (ci < aP && (uint32_t)(rbase + ci) < un)
            Pay<V>::st(cr_pre, rbase + ci, unite(pre_t, pu[j]));
    }
    // Closes of blends opened in an earlier thread of this partition.  A
    // wave gathers its lanes' closes into LDS and then takes them 64 at a
    // time, one per lane, so the union-tree queries do not run as many
    // rounds as the busiest lane has closes; closes past the buffer stay
    // with their lane and are taken one per round.
    {
        constexpr int DCAP = ResolveSmem<BOXES, V, KK>::DCAP;
        const int nd = (int)__popc(dloc);
        int wnd;
        const int doff = wave_excl_scan(nd, AddOp{}, 0, &wnd);
        const int wb = wid * DCAP;
        int k = doff;
#pragma unroll
        for (int j = 0; j < KK; ++j) {
            if (!((dloc >> j) & 1u)) continue;
            if (k < DCAP) {
                sm.e.d.item[wb + k] = make_int2((int)(dfw[j] | ((uint32_t)j << 24)), t);
                sm.e.d.pre[wb + k] = pu[j];
                dloc &= ~(1u << j);
            }
            ++k;
        }
        asm volatile("" ::: "memory");  // a wave's LDS accesses complete in order
        const int nbuf = min(wnd, DCAP);
        for (int i0 = 0; i0 < nbuf; i0 += WAVE) {
            const int i = i0 + lane;
            if (i >= nbuf) continue;
            const int2 it2 = sm.e.d.item[wb + i];
            const V pre = sm.e.d.pre[wb + i];
            const uint32_t w = (uint32_t)it2.x & 0xFFFFFFu;
            const int j = (int)((uint32_t)it2.x >> 24), tt = it2.y;
            const int s = (int)(w & 0x1FFu) - 1, pos = (int)((w >> 9) & 7u), ent = (int)(w >> 12);
            const V u = unite(unite(sm.cx[ent], uniontree_inner<V, WW>(ut, s + 1, tt - 1)), pre);
            sink.emit(p0 + (uint32_t)tt * KK + j, u);
            sink.emit(p0 + (uint32_t)s * KK + pos, u);
        }
    }
    for (int it = 0; it < KK && __ballot(dloc != 0); ++it) {
        if (!dloc) continue;
        const int j = __builtin_ctz(dloc);
        dloc &= dloc - 1;
        uint32_t w = dfw[0];
        V pre = pu[0];
        uint32_t jm = 1u << j;
        asm("" : "+v"(jm));  // opaque: the selects stay selects, not an indexed load
#pragma unroll
        for (int q = 1; q < KK; ++q) {
            w = ((jm >> q) & 1u) ? dfw[q] : w;
            pre = vsel(((jm >> q) & 1u) != 0, pu[q], pre);
        }
        const int s = (int)(w & 0x1FFu) - 1, pos = (int)((w >> 9) & 7u), ent = (int)(w >> 12);
        const V u = unite(unite(sm.cx[ent], uniontree_inner<V, WW>(ut, s + 1, t - 1)), pre);
        sink.emit(g0 + j, u);
        sink.emit(p0 + (uint32_t)s * KK + pos, u);
    }
    // surviving blend opens: union from the open to the end of the partition
    {
        const int baseP = myp.z;
        int jj = 0;
#pragma unroll
        for (int p = 0; p < KK; ++p) {
            if (!((wk.umask >> p) & 1u)) continue;
            const int L = base + 1 + jj;
            const int e = ub + jj;
            ++jj;
            if (L > sufmin || ks[p] != BBLEND) continue;
            const int slot = L - baseP - 1;
            if (slot < 0 || slot >= T || e > T) continue;
            Pay<V>::st(U_suf, p0 + (uint32_t)slot, unite(sm.cx[e], suf_t));
        }
    }
    if (t == 0) Pay<V>::st(ptot, P, all);
}

// ------------------------------------------------ range unions over partitions
// Blocks of UB partitions: inclusive prefix and suffix unions inside each
// block, block totals, and an in-block sparse table (level l at partition q
// holds the union of partitions q .. q+2^l-1, clipped to the block).
constexpr int UBL = 8;  // log2(UB)
template <class V>
__global__ __launch_bounds__(UB) void k_ublocks(const void *__restrict__ ptot, int64_t M,
                                                void *__restrict__ upre, void *__restrict__ usuf,
                                                void *__restrict__ btot, void *__restrict__ spb) {
    __shared__ V sh[UB / WAVE];
    __shared__ V lv[UB];
    const int t = threadIdx.x;
    const int64_t B = blockIdx.x;
    const int64_t P = B * UB + t;
    const int64_t Pr = B * UB + (UB - 1 - t);
    const V v = P < M ? Pay<V>::ld(ptot, P) : Pay<V>::empty();
    const V vr = Pr < M ? Pay<V>::ld(ptot, Pr) : Pay<V>::empty();
    V tot, tot2;
    const V ex = block_excl_scan<UB / WAVE>(v, UniteOp{}, Pay<V>::empty(), sh, &tot);
    const V exr = block_excl_scan<UB / WAVE>(vr, UniteOp{}, Pay<V>::empty(), sh, &tot2);
    if (P < M) Pay<V>::st(upre, P, unite(ex, v));
    if (Pr < M) Pay<V>::st(usuf, Pr, unite(exr, vr));
    if (t == 0) Pay<V>::st(btot, B, tot);
    V cur = v;
    lv[t] = cur;
    if (P < M) Pay<V>::st(spb, P, cur);
    for (int l = 1; l < UBL; ++l) {
        __syncthreads();
        const int h = 1 << (l - 1);
        if (t + h < UB) cur = unite(cur, lv[t + h]);
        __syncthreads();
        lv[t] = cur;
        if (P < M) Pay<V>::st(spb, (int64_t)l * M + P, cur);
    }
}

// Sparse table over block totals: level l holds unions of 2^l blocks.
// Level 0 is the block totals themselves (the first nb entries of sp).
template <class V>
__global__ __launch_bounds__(1024) void k_usparse(void *__restrict__ sp, int64_t nb, int levels) {
    for (int l = 1; l < levels; ++l) {
        const int64_t half = (int64_t)1 << (l - 1);
        for (int64_t b = threadIdx.x; b < nb; b += 1024) {
            V v = Pay<V>::ld(sp, (l - 1) * nb + b);
            if (b + half < nb) v = unite(v, Pay<V>::ld(sp, (l - 1) * nb + b + half));
            Pay<V>::st(sp, l * nb + b, v);
        }
        __syncthreads();
    }
}

template <class V, class SINK, int U>
__global__ __launch_bounds__(W) void k_cross(const int *__restrict__ crtot, int64_t n,
                                             const int64_t *__restrict__ off, int64_t S,
                                             const int32_t *__restrict__ U_idx,
                                             const void *__restrict__ U_suf,
                                             const int32_t *__restrict__ cr_slot,
                                             const int32_t *__restrict__ cr_c,
                                             const void *__restrict__ cr_pre,
                                             const void *__restrict__ upre,
                                             const void *__restrict__ usuf,
                                             const void *__restrict__ sp,
                                             const void *__restrict__ spb, int64_t M, int64_t nb,
                                             int32_t *__restrict__ match, SINK sink) {
    // One thread per close record: a close whose open lies in an earlier
    // partition.  Both rows and both match entries of the pair are written
    // here, so consecutive records write consecutive rows.  A clip pair's box
    // is the open's full clip context, which k_resolve put in the record
    // (read densely here, whatever the kinds of the neighbouring records); a
    // blend pair's is the union of the open's suffix, the whole partitions
    // between and the close's prefix (the record's payload).  Records are dense and their count is on the device.  A
    // workgroup takes contiguous chunks of U*W records, U per thread; after
    // the records themselves every load is issued at once (unused lanes read
    // entry 0 and discard it).
    const int64_t total = min((int64_t)*crtot, n);  // at most one record per element
    for (int64_t c0 = (int64_t)blockIdx.x * (U * W); c0 < total; c0 += (int64_t)gridDim.x * (U * W)) {
        const int64_t r0 = c0 + threadIdx.x;
        int64_t sl[U], cc[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t r = r0 + q * W;
            sl[q] = r < total ? cr_slot[r] : -1;
            cc[q] = r < total ? (int64_t)(uint32_t)cr_c[r] : -1;
        }
        bool bl[U];  // blend pair (the close record's top bit)
#pragma unroll
        for (int q = 0; q < U; ++q) {
            bl[q] = cc[q] >= 0 && (cc[q] & 0x80000000ll);
            if (cc[q] >= 0) cc[q] &= 0x7FFFFFFFll;
        }
        int32_t ui[U];
        V part[U], cl[U], x1[U], x2[U], x3[U], x4[U];
        bool ok[U], ne[U], mid[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t r = r0 + q * W;
            ok[q] = sl[q] >= 0 && sl[q] < M * T && cc[q] >= 0 && cc[q] < n && sl[q] / T < cc[q] / T;
            const int64_t s0 = ok[q] ? sl[q] : 0;
            ui[q] = U_idx[s0];
            // the record's payload: a clip pair's box (the open's full
            // context), or a blend close's prefix union; a blend pair also
            // needs the open's suffix union (other lanes read entry 0)
            const V pre = Pay<V>::ld(cr_pre, ok[q] ? r : 0);
            cl[q] = pre;
            part[q] = unite(Pay<V>::ld(U_suf, bl[q] ? s0 : 0), pre);
            // whole partitions strictly between: [a, b]
            const int64_t a = ok[q] && bl[q] ? sl[q] / T + 1 : 1, b = ok[q] && bl[q] ? cc[q] / T - 1 : 0;
            ne[q] = a <= b;
            const int64_t ba = a / UB, bb = b / UB;
            const bool same = ba == bb;
            const int64_t len = ne[q] ? b - a + 1 : 1;
            const int ls = min(63 - __clzll((unsigned long long)len), UBL - 1);
            const void *p1 = same ? spb : usuf;
            const void *p2 = same ? spb : upre;
            const int64_t i1 = !ne[q] ? 0 : same ? ls * M + a : a;
            const int64_t i2 = !ne[q] ? 0 : same ? ls * M + b - ((int64_t)1 << ls) + 1 : b;
            const int64_t l0 = ba + 1, l1 = bb - 1;
            mid[q] = ne[q] && !same && l0 <= l1;
            const int lm = mid[q] ? 63 - __clzll((unsigned long long)(l1 - l0 + 1)) : 0;
            const int64_t i3 = mid[q] ? lm * nb + l0 : 0;
            const int64_t i4 = mid[q] ? lm * nb + l1 - ((int64_t)1 << lm) + 1 : 0;
            x1[q] = Pay<V>::ld(p1, i1);
            x2[q] = Pay<V>::ld(p2, i2);
            x3[q] = Pay<V>::ld(sp, i3);
            x4[q] = Pay<V>::ld(sp, i4);
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t o = (int64_t)((uint32_t)ui[q] & ~BLEND_BIT);
            if (!ok[q] || o >= n) continue;
            V u;
            if (bl[q]) {
                u = part[q];
                if (ne[q]) u = unite(u, unite(x1[q], x2[q]));
                if (mid[q]) u = unite(u, unite(x3[q], x4[q]));
            } else {
                u = canon(cl[q]);
            }
            sink.emit(o, u);
            sink.emit(cc[q], u);
            if (match) {
                const int64_t soff = off ? off[scene_of(off, S, cc[q])] : 0;
                match[o] = (int32_t)(cc[q] - soff);
                match[cc[q]] = (int32_t)(o - soff);
            }
        }
    }
}

// ------------------------------------------------------------------ sinks
// Forward: node boxes are written out.
struct SinkOut {
    static constexpr bool kPos = false;  // rows go to element indices
    float4 *out;
    __device__ __forceinline__ void emit(int64_t i, const Box &v) const { st_box(out, i, v); }
};

// Stream front end: rows of the extracted sequence go to their elements'
// stream positions (idx[i] < ns; any other value is dropped, which only
// stale workspace entries of malformed input can hold).
struct SinkScatter {
    // k_resolve reads a thread's own positions with its inputs (pos) and
    // writes those rows with emit_at, so no store waits on a position load
    static constexpr bool kPos = true;
    float4 *out;
    const int32_t *idx;
    uint32_t ns;
    __device__ __forceinline__ uint32_t pos(int64_t i) const { return (uint32_t)idx[i]; }
    __device__ __forceinline__ void emit_at(uint32_t j, const Box &v) const {
        if (j < ns) st_box(out, j, v);
    }
    __device__ __forceinline__ void emit(int64_t i, const Box &v) const { emit_at(pos(i), v); }
};

// Composition down the tree: each row's transform is written out.
struct SinkAff {
    static constexpr bool kPos = false;
    void *out;
    __device__ __forceinline__ void emit(int64_t i, const Aff &v) const { Pay<Aff>::st(out, i, v); }
};

// Backward: each coordinate of a non-EMPTY output row routes q(g) to its
// attaining input element.  A row's own coordinates are flagged in a
// per-row mask (no atomics); every other route is an exact 64-bit atomic add.
// q(g) = g * 2^32 rounded half-to-even to an integer, defined for |g| < 2^31;
// a routed g outside that range (or NaN) raises GRAD_RANGE instead.
constexpr uint32_t ST_GRAD_RANGE = 16u;
__device__ __forceinline__ bool grad_in_range(float g) { return fabsf(g) < 2147483648.0f; }

struct SinkGrad {
    static constexpr bool kPos = false;
    const float4 *g;
    unsigned long long *acc;  // [n][4] two's-complement sums on the 2^-32 grid
    uint8_t *selfm;           // [n] bit c: row i routes coordinate c to itself
    int64_t n;
    uint32_t *status;
    __device__ __forceinline__ void emit(int64_t i, const BoxS &v) const {
        uint32_t m = 0;
        bool bad = false;
        if (boxs_nonempty(v)) {
            const float4 gv = g[i];
            const float gc[4] = {gv.x, gv.y, gv.z, gv.w};
            const int32_t sc[4] = {boxs_src(v, 0), boxs_src(v, 1), boxs_src(v, 2), boxs_src(v, 3)};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t s = sc[c];
                if (s < 0 || s >= n) continue;
                bad |= !grad_in_range(gc[c]);
                if (s == i) {
                    m |= 1u << c;
                } else if (gc[c] != 0.0f && grad_in_range(gc[c])) {
                    const long long q = __double2ll_rn((double)gc[c] * 4294967296.0);
                    atomicAdd(acc + 4 * s + c, (unsigned long long)q);
                }
            }
        }
        if (bad) atomicOr(status, ST_GRAD_RANGE);
        selfm[i] = (uint8_t)m;
    }
};

__global__ void k_zero_u64(unsigned long long *p, int64_t cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0ull;
}

// grad_in = RNE_fp32(acc + own q(g)) * 2^-32; the integer sums wrap modulo
// 2^64, so only the final sum has to fit in an int64
__global__ void k_grad_final(const float4 *__restrict__ g, const unsigned long long *__restrict__ acc,
                             const uint8_t *__restrict__ selfm, float4 *__restrict__ gin, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t m = selfm[i];
    const float4 gv = g[i];
    const float gc[4] = {gv.x, gv.y, gv.z, gv.w};
    float r[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        unsigned long long s = acc[4 * i + c];
        if (((m >> c) & 1u) && grad_in_range(gc[c]))
            s += (unsigned long long)__double2ll_rn((double)gc[c] * 4294967296.0);
        r[c] = __ll2float_rn((long long)s) * 0x1p-32f;
    }
    gin[i] = make_float4(r[0], r[1], r[2], r[3]);
}


// ------------------------------------------------- draw-object stream front end
// The tree's elements (tags 0..4) are extracted from a stream that also
// holds elements outside the tree (tag 5) by stream compaction, a prefix-sum
// application (Introduction); the pipeline then runs on the extracted
// sequence only.  Blocks of CT stream elements: count, an exclusive scan of
// the block counts, scatter.  Inside a block, element order is round q
// (1024 elements each), then thread, then the thread's 4 consecutive
// elements, so each round is one 16-byte load per thread.  The pipeline
// writes rows straight to stream positions; partners are translated after.
constexpr int CW = 256;          // threads per compaction block
constexpr int CR = 8;            // rounds of 4 elements per thread
constexpr int CT = CW * 4 * CR;  // stream elements per block
constexpr uint32_t TAG_OTHER = 5;
// Word 3 of a raw (stride 0) buffer resource on gfx9-family chips: 32-bit
// data format, no swizzle; out-of-range offsets read as zero.
constexpr int BUF_DWORD3 = 0x00020000;

// Tags of round q for this thread; past the end reads as TAG_OTHER.
__device__ __forceinline__ void load_tags4(const uint32_t *tag, int64_t n, int64_t e0,
                                           uint32_t (&v)[4]) {
    if (e0 + 4 <= n && ((uintptr_t)tag & 15u) == 0) {
        const uint4 x = *reinterpret_cast<const uint4 *>(tag + e0);
        v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = e0 + c < n ? tag[e0 + c] : TAG_OTHER;
    }
}

__global__ __launch_bounds__(CW) void k_cmp_count(const uint32_t *__restrict__ tag, int64_t n,
                                                  int *__restrict__ cnt,
                                                  uint32_t *__restrict__ status) {
    __shared__ int sh[CW / WAVE];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wid = t >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * CT;
    uint32_t v[CR][4];
#pragma unroll
    for (int q = 0; q < CR; ++q) load_tags4(tag, n, b0 + q * (CW * 4) + 4 * t, v[q]);
    int c = 0;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < CR; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c += v[q][j] <= 4u ? 1 : 0;
            bad |= v[q][j] > TAG_OTHER;
        }
    }
    if (bad) flag(status, nullptr, 1, 0, ST_BAD_KIND);
    int wt;
    wave_excl_scan(c, AddOp{}, 0, &wt);
    if (lane == 0) sh[wid] = wt;
    __syncthreads();
    if (t == 0) {
        int tot = 0;
#pragma unroll
        for (int w = 0; w < CW / WAVE; ++w) tot += sh[w];
        cnt[blockIdx.x] = tot;
    }
}

// One workgroup: exclusive scan of the nblk block counts in place, in
// chunks of 1024 threads x 8 counts; the total goes to *m.
__global__ __launch_bounds__(1024) void k_cmp_scan(int *__restrict__ cnt, int64_t nblk,
                                                   int64_t *__restrict__ m) {
    __shared__ int sh[1024 / WAVE];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nblk; c0 += 1024 * 8) {
        int v[8], s = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t i = c0 + (int64_t)t * 8 + j;
            v[j] = i < nblk ? cnt[i] : 0;
            s += v[j];
        }
        int tot;
        const int ex = block_excl_scan<1024 / WAVE>(s, AddOp{}, 0, sh, &tot);
        int64_t run = carry + ex;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t i = c0 + (int64_t)t * 8 + j;
            if (i < nblk) cnt[i] = (int)run;
            run += v[j];
        }
        carry += tot;
    }
    if (t == 0) *m = carry;
}

// Scatter the tree elements of each block to their extracted positions:
// kind, stream index, and the box of leaves and clip opens (the only rows
// the pipeline reads).
__global__ __launch_bounds__(CW) void k_cmp_scatter(const uint32_t *__restrict__ tag,
                                                    const float4 *__restrict__ box, int64_t n,
                                                    const int *__restrict__ boff,
                                                    uint32_t *__restrict__ ckind,
                                                    float4 *__restrict__ cbox,
                                                    int32_t *__restrict__ cidx) {
    __shared__ int grp[CR * (CW / WAVE)];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wid = t >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * CT;
    uint32_t v[CR][4];
#pragma unroll
    for (int q = 0; q < CR; ++q) load_tags4(tag, n, b0 + q * (CW * 4) + 4 * t, v[q]);
    int lex[CR];  // tree elements of earlier lanes of this wave, per round
#pragma unroll
    for (int q = 0; q < CR; ++q) {
        int c = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) c += v[q][j] <= 4u ? 1 : 0;
        int wt;
        lex[q] = wave_excl_scan(c, AddOp{}, 0, &wt);
        if (lane == 0) grp[q * (CW / WAVE) + wid] = wt;
    }
    __syncthreads();
    // boxes through a buffer resource over this block's rows: a lane that
    // needs no box passes an out-of-range offset, which reads zero without a
    // memory access, so the gathers need no branches (and no waits between)
    const int64_t rem = n - b0;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(box + b0), (short)0, (int)((rem < CT ? rem : CT) * (int64_t)sizeof(float4)),
        BUF_DWORD3);
    float4 bq[CR][4];  // every gather is issued before the first store
#pragma unroll
    for (int q = 0; q < CR; ++q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool need = v[q][j] == LEAF || v[q][j] == BCLIP;
            const int off = need ? (q * (CW * 4) + 4 * t + j) * (int)sizeof(float4) : -1;
            bq[q][j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        }
    }
    const int64_t base = boff[blockIdx.x];
    int rb = 0;  // tree elements in the rounds before this one
#pragma unroll
    for (int q = 0; q < CR; ++q) {
        int o = rb;  // ... plus those of this round's earlier waves
#pragma unroll
        for (int w = 0; w < CW / WAVE; ++w) {
            const int gw = grp[q * (CW / WAVE) + w];
            if (w < wid) o += gw;
            rb += gw;
        }
        int64_t d = base + o + lex[q];
        const int64_t e0 = b0 + q * (CW * 4) + 4 * t;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t k = v[q][j];
            if (k > 4u) continue;
            ckind[d] = k;
            cidx[d] = (int32_t)(e0 + j);
            if (k == LEAF || k == BCLIP) cbox[d] = bq[q][j];
            ++d;
        }
    }
}

// Partners of the extracted sequence, translated to stream positions; four
// per thread and round so that the dependent gathers overlap.
__global__ void k_stream_match(const int32_t *__restrict__ cmatch,
                               const int32_t *__restrict__ cidx, const int64_t *__restrict__ m,
                               int32_t *__restrict__ match) {
    const int64_t mm = *m;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c0 < mm; c0 += 4 * stride) {
        int32_t p[4], i[4], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t c = c0 + u * stride;
            p[u] = c < mm ? cmatch[c] : -1;
            i[u] = c < mm ? cidx[c] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = (p[u] >= 0 && p[u] < mm) ? cidx[p[u]] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u * stride < mm) match[i[u]] = q[u];
    }
}

// --------------------------------------- fp32 transforms by pointer jumping
// A monoid whose products round: 2-D affine transforms in fp32, composed
// down the tree in the order of pointer jumping over the opens (section
// "Parallel bounding boxes", Clips): each round every open replaces its
// value v by (value at its pointer) . v and its pointer by the pointer's
// pointer, all from the previous round's arrays.  Every product and every
// sum rounds on its own (no fused multiply-add), in the order written in
// f32_mul, so the result is defined bit for bit.
struct F32Aff {
    float a, b, c, d, e, f;
};
__device__ __forceinline__ F32Aff f32_id() { return {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f}; }
// p . q (q applied first)
__device__ __forceinline__ F32Aff f32_mul(const F32Aff &p, const F32Aff &q) {
#pragma clang fp contract(off)
    return {__fadd_rn(__fmul_rn(p.a, q.a), __fmul_rn(p.b, q.d)),
            __fadd_rn(__fmul_rn(p.a, q.b), __fmul_rn(p.b, q.e)),
            __fadd_rn(__fadd_rn(__fmul_rn(p.a, q.c), __fmul_rn(p.b, q.f)), p.c),
            __fadd_rn(__fmul_rn(p.d, q.a), __fmul_rn(p.e, q.d)),
            __fadd_rn(__fmul_rn(p.d, q.b), __fmul_rn(p.e, q.e)),
            __fadd_rn(__fadd_rn(__fmul_rn(p.d, q.c), __fmul_rn(p.e, q.f)), p.f)};
}
// rows of 24 bytes, 8-byte aligned
__device__ __forceinline__ F32Aff f32_ld(const float *base, int64_t i) {
    const float2 *q = (const float2 *)base + 3 * i;
    const float2 x = q[0], y = q[1], z = q[2];
    return {x.x, x.y, y.x, y.y, z.x, z.y};
}
__device__ __forceinline__ void f32_st(float *base, int64_t i, const F32Aff &v) {
    float2 *q = (float2 *)base + 3 * i;
    q[0] = make_float2(v.a, v.b);
    q[1] = make_float2(v.c, v.d);
    q[2] = make_float2(v.e, v.f);
}
constexpr int XJ_ROUNDS = 32;  // flag words: flags[r] = 1 when round r+1 has work

// every open: its own transform and a pointer to its enclosing open (pm);
// other elements hold the identity and no pointer
__global__ void k_xj_init(const uint32_t *__restrict__ kind, const float *__restrict__ xf,
                          const int32_t *__restrict__ pm, int64_t n, float *__restrict__ val,
                          int32_t *__restrict__ ptr, uint32_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool live = false;
    if (i < n) {
        const uint32_t k = kind[i];
        const bool open = k == BCLIP || k == BBLEND;
        const int32_t p = open ? pm[i] : -1;
        f32_st(val, i, open ? f32_ld(xf, i) : f32_id());
        ptr[i] = p;
        live = p >= 0;
    }
    if (__ballot(live) && (threadIdx.x & (WAVE - 1)) == 0) flags[0] = 1u;  // every writer stores 1
}

// round r (>= 1): runs only if round r-1 left a pointer
__global__ void k_xj_round(int r, const int32_t *__restrict__ ptr_in, const float *__restrict__ val_in,
                           int32_t *__restrict__ ptr_out, float *__restrict__ val_out, int64_t n,
                           uint32_t *__restrict__ flags) {
    if (!flags[r - 1]) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool live = false;
    if (i < n) {
        const int32_t p = ptr_in[i];
        F32Aff v = f32_ld(val_in, i);
        int32_t np = -1;
        if (p >= 0 && p < n) {
            v = f32_mul(f32_ld(val_in, p), v);  // the enclosing part first
            np = ptr_in[p];
        }
        f32_st(val_out, i, v);
        ptr_out[i] = np;
        live = np >= 0;
    }
    if (__ballot(live) && (threadIdx.x & (WAVE - 1)) == 0) flags[r] = 1u;
}

// results from the buffer the last executed round wrote: an open's own
// value, a leaf's or close's the value of pm[i] (its enclosing or own open)
__global__ void k_xj_out(const uint32_t *__restrict__ kind, const int32_t *__restrict__ pm,
                         const float *__restrict__ val0, const float *__restrict__ val1, int64_t n,
                         float *__restrict__ out, const uint32_t *__restrict__ flags, int rounds) {
    int last = 0;
    for (int r = 1; r <= rounds && flags[r - 1]; ++r) last = r;
    const float *val = (last & 1) ? val1 : val0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = kind[i];
    const int32_t p = pm[i];
    const bool open = k == BCLIP || k == BBLEND;
    f32_st(out, i, open ? f32_ld(val, i) : (p >= 0 && p < n) ? f32_ld(val, p) : f32_id());
}

// ------------------------------- fp32 transforms multiplied up the tree
// Every open (and its close) gets the ordered product of the transforms of
// the leaves strictly between them, leftmost leaf leftmost.  Products round,
// so the grouping is fixed by a segment tree over positions: leaf node N+i
// holds element i's transform if it is a leaf, node v = node 2v . node 2v+1
// (a side without leaves leaves the other unchanged), and a range is read
// bottom-up, left boundary nodes folded left to right, right boundary nodes
// right to left, then the two joined.  A node without leaves holds NONE, a
// NaN bit pattern no finite input or fp32 operation produces.
constexpr uint32_t UP_NONE = 0xFFFFFFFFu;
__device__ __forceinline__ bool up_none(const F32Aff &v) { return __float_as_uint(v.a) == UP_NONE; }
__device__ __forceinline__ F32Aff up_none_val() {
    const float x = __uint_as_float(UP_NONE);
    return {x, x, x, x, x, x};
}
__device__ __forceinline__ F32Aff up_comb(const F32Aff &a, const F32Aff &b) {
    return up_none(a) ? b : up_none(b) ? a : f32_mul(a, b);
}

__global__ void k_up_leaves(const uint32_t *__restrict__ kind, const float *__restrict__ xf, int64_t n,
                            int64_t N, float *__restrict__ node) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    f32_st(node, N + i, (i < n && kind[i] == LEAF) ? f32_ld(xf, i) : up_none_val());
}

// nodes [h, 2h) from their children
__global__ void k_up_level(int64_t h, float *__restrict__ node) {
    const int64_t v = h + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= 2 * h) return;
    f32_st(node, v, up_comb(f32_ld(node, 2 * v), f32_ld(node, 2 * v + 1)));
}

__global__ void k_up_query(const uint32_t *__restrict__ kind, const float *__restrict__ xf,
                           const int32_t *__restrict__ match, int64_t n, int64_t N,
                           const float *__restrict__ node, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = kind[i];
    const int64_t m = match[i];
    if (k == LEAF) {
        f32_st(out, i, f32_ld(xf, i));
        return;
    }
    if (!is_open(k) || m <= i || m >= n) {
        if (!(is_close(k) && m >= 0 && m < i)) f32_st(out, i, f32_id());  // malformed: unspecified
        return;
    }
    F32Aff L = up_none_val(), R = up_none_val();
    int64_t l = i + 1 + N, r = m + N;  // leaves (i, m): [i+1, m-1]
    while (l < r) {
        if (l & 1) L = up_comb(L, f32_ld(node, l++));
        if (r & 1) R = up_comb(f32_ld(node, --r), R);
        l >>= 1;
        r >>= 1;
    }
    F32Aff q = up_comb(L, R);
    if (up_none(q)) q = f32_id();
    f32_st(out, i, q);
    f32_st(out, m, q);
}

// ----------------------------------------------------------------- driver
hipEvent_t g_prof_before = nullptr, g_prof_after = nullptr;

static inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

FwdLayout fwd_layout(int64_t n, int64_t S, size_t vbytes, bool grad) {
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
    L.bagg = take(sizeof(int4) * ((Mp + SB - 1) / SB + 1));
    L.crbase = take(sizeof(int) * M);
    L.crtot = take(sizeof(int) * 4);
    L.jptr0 = take(sizeof(int32_t) * M);
    L.jptr1 = take(sizeof(int32_t) * M);
    L.jval0 = take(vbytes * M);
    L.jval1 = take(vbytes * M);
    L.U_idx = take(sizeof(int32_t) * M * T);
    L.U_cum = take(vbytes * M * T);
    L.U_suf = take(vbytes * M * T);
    L.cr_slot = take(sizeof(int32_t) * M * T);
    L.cr_c = take(sizeof(int32_t) * M * T);
    L.cr_pre = take(vbytes * M * T);
    L.runs = take(sizeof(int4) * M * RMAX);
    L.rhead = take(sizeof(int4) * M);
    L.ptot = take(vbytes * M);
    L.upre = take(vbytes * M);
    L.usuf = take(vbytes * M);
    L.sp = take(vbytes * nb * lv);
    L.spb = take(vbytes * M * UBL);
    L.status = take(sizeof(uint32_t) * (S > 0 ? S : 1));
    L.offflag = take(sizeof(uint32_t));
    if (grad) {
        L.acc = take(sizeof(unsigned long long) * 4 * (n > 0 ? n : 1));
        L.selfm = take(n > 0 ? n : 1);
    }
    L.total = o;
    return L;
}

// Launch shapes that a variant may change: only the forward box path
// (tb_bbox, tb_bbox_batched) and matching alone have more than one; every
// other payload runs the default.
template <bool BOXES, class V, class SINK>
constexpr bool kTunable = !BOXES || (std::is_same<V, Box>::value && std::is_same<SINK, SinkOut>::value);

template <bool BOXES, class V, class SINK, int KD, bool BRK>
static void launch_reduce(int64_t M, hipStream_t st, const uint32_t *kind, const float4 *box, int64_t n,
                          const int64_t *off, int64_t S, int4 *pinfo, int32_t *U_idx, void *U_cum,
                          const int64_t *n_dyn, uint32_t *zst) {
    if (off)
        k_reduce<BOXES, V, KD, BRK, true><<<(unsigned)M, T / KD, 0, st>>>(kind, box, n, off, S, pinfo, U_idx,
                                                                         U_cum, n_dyn, zst);
    else
        k_reduce<BOXES, V, KD, BRK, false><<<(unsigned)M, T / KD, 0, st>>>(kind, box, n, off, S, pinfo, U_idx,
                                                                          U_cum, n_dyn, zst);
}

// BRK: the kinds are typed bracket tokens (matching alone)
template <bool BOXES, class V, class SINK, bool BRK = false>
static hipError_t run_pipeline(const uint32_t *kind, const float4 *box, int64_t n,
                               const int64_t *off, int64_t S, int32_t *match, int32_t *pm,
                               SINK sink, char *w, const FwdLayout &L, uint32_t *status,
                               hipStream_t st, const int64_t *n_dyn = nullptr,
                               Variant var = Variant{}, uint32_t *zst = nullptr) {
    if (!kTunable<BOXES, V, SINK> || !variant_ok(var)) var = default_variant(BOXES);
    // Parents (pm) take a lookup at every element whose thread-local stack is
    // empty; with 8 elements per thread that walk ran about 20% slower than
    // with 4 on 2^27-element scenes, so such calls use 4 whatever the variant.
    if (!BOXES && pm && var.kr == 8) var.kr = 4;
    const int64_t M = L.M;
    int4 *pinfo = (int4 *)(w + L.pinfo);
    int4 *part = (int4 *)(w + L.part);
    int *mtree = (int *)(w + L.mtree);
    int *crbase = (int *)(w + L.crbase);
    int *crtot = (int *)(w + L.crtot);
    int32_t *U_idx = (int32_t *)(w + L.U_idx);
    void *U_cum = w + L.U_cum;
    // elements per thread of the reduce
    if (var.kd == 8)
        launch_reduce<BOXES, V, SINK, 8, BRK>(M, st, kind, box, n, off, S, pinfo, U_idx, U_cum, n_dyn, zst);
    else
        launch_reduce<BOXES, V, SINK, 4, BRK>(M, st, kind, box, n, off, S, pinfo, U_idx, U_cum, n_dyn, zst);
    {
        int4 *bagg = (int4 *)(w + L.bagg);
        const int64_t nbk = (M + SB - 1) / SB;
        const int64_t nbt = (L.Mp + SB - 1) / SB;
        const bool single = nbt == 1;  // all partitions (and tree leaves) in one block
        if (!single) {
            k_spine_blocks<<<(unsigned)nbk, SB, 0, st>>>(pinfo, M, bagg);
            k_spine_top<<<1, SB, 0, st>>>(bagg, nbk, off, S, n, status, crtot);
        }
        k_spine_apply<<<(unsigned)nbt, SB, 0, st>>>(pinfo, M, bagg, part, mtree, L.Mp, crbase, single,
                                                    off, S, n, status, crtot);
        if (L.Mp > SB) k_spine_treetop<<<1, SB, 0, st>>>(mtree, L.Mp);
    }
    int32_t *jp[2] = {(int32_t *)(w + L.jptr0), (int32_t *)(w + L.jptr1)};
    void *jv[2] = {w + L.jval0, w + L.jval1};
    const unsigned gM = (unsigned)((M + 255) / 256);
    int4 *runs = (int4 *)(w + L.runs);
    int4 *rhead = (int4 *)(w + L.rhead);
    int rounds = 0;
    while (((int64_t)1 << rounds) < M) ++rounds;
    int cur = 0;
    if (M <= JS) {  // links, jumping and runs in one launch
        k_link_small<BOXES, V><<<1, JS, 0, st>>>(pinfo, part, M, mtree, L.Mp, U_cum, jp[0], jv[0],
                                                 rounds, runs, rhead);
    } else {
        k_spine_link<BOXES, V><<<gM, 256, 0, st>>>(pinfo, part, M, mtree, L.Mp, U_cum, jp[0], jv[0]);
        if (BOXES) {
            for (int64_t reach = 1; reach < M; reach *= JH) {  // reach: owners covered so far
                k_jump<V><<<gM, 256, 0, st>>>(jp[cur], jv[cur], jp[cur ^ 1], jv[cur ^ 1], M);
                cur ^= 1;
            }
        }
        k_runs<<<gM, 256, 0, st>>>(pinfo, part, M, runs, rhead);
    }
    void *U_suf = w + L.U_suf;
    int32_t *cr_slot = (int32_t *)(w + L.cr_slot);
    int32_t *cr_c = (int32_t *)(w + L.cr_c);
    void *cr_pre = w + L.cr_pre;
    void *ptot = w + L.ptot;
    const bool prof = g_prof_before && g_prof_after;
    if (prof) (void)hipEventRecord(g_prof_before, st);
    // elements per thread of the main pass (more elements per thread share
    // the partition-level steps among fewer threads)
    auto resolve = [&](auto kr) {
        constexpr int KR = decltype(kr)::value;
        if (off)
            k_resolve<BOXES, V, SINK, KR, BRK, true><<<(unsigned)M, T / KR, 0, st>>>(
                kind, box, n, off, S, pinfo, part, runs, rhead, jv[cur], U_idx, U_cum, U_suf, crbase,
                cr_slot, cr_c, cr_pre, ptot, match, pm, sink, status, n_dyn);
        else
            k_resolve<BOXES, V, SINK, KR, BRK, false><<<(unsigned)M, T / KR, 0, st>>>(
                kind, box, n, off, S, pinfo, part, runs, rhead, jv[cur], U_idx, U_cum, U_suf, crbase,
                cr_slot, cr_c, cr_pre, ptot, match, pm, sink, status, n_dyn);
    };
    if constexpr (kTunable<BOXES, V, SINK>) {
        if (var.kr == 8)
            resolve(std::integral_constant<int, 8>{});
        else
            resolve(std::integral_constant<int, 4>{});
    } else {
        resolve(std::integral_constant<int, K>{});
    }
    if (prof) (void)hipEventRecord(g_prof_after, st);
    if (BOXES) {
        void *upre = w + L.upre;
        void *usuf = w + L.usuf;
        void *sp = w + L.sp;
        void *spb = w + L.spb;
        if (Pay<V>::kUnions) {
            k_ublocks<V><<<(unsigned)L.nb, UB, 0, st>>>(ptot, M, upre, usuf, sp, spb);
            if (L.levels > 1) k_usparse<V><<<1, 1024, 0, st>>>(sp, L.nb, L.levels);
        }
        const int64_t gx = min((int64_t)(n + W - 1) / W, (int64_t)256 * 32);
        auto cross = [&](auto u) {
            constexpr int U = decltype(u)::value;
            k_cross<V, SINK, U><<<(unsigned)gx, W, 0, st>>>(crtot, n, off, S, U_idx, U_suf,
                                                            cr_slot, cr_c, cr_pre, upre, usuf, sp, spb,
                                                            M, L.nb, match, sink);
        };
        if constexpr (kTunable<BOXES, V, SINK>) {
            if (var.cu == 2)
                cross(std::integral_constant<int, 2>{});
            else if (var.cu == 8)
                cross(std::integral_constant<int, 8>{});
            else
                cross(std::integral_constant<int, 4>{});
        } else {
            cross(std::integral_constant<int, sizeof(V) <= 16 ? 4 : 2>{});
        }
    }
    return hipGetLastError();
}

// Clears the status words (and the offsets flag).  With `defer` (one scene,
// n > 0) nothing is launched: the pipeline's first kernel clears the word.
static uint32_t *prep_status(char *w, const FwdLayout &L, const int64_t *off, int64_t S,
                             int64_t n, uint32_t *status, hipStream_t st, bool defer = false) {
    const int64_t nstat = off ? S : 1;
    if (!status) status = (uint32_t *)(w + L.status);
    if (defer && !off && n > 0) return status;
    uint32_t *flagw = (uint32_t *)(w + L.offflag);
    k_zero_status<<<(unsigned)((nstat + 255) / 256), 256, 0, st>>>(status, nstat, flagw);
    if (off) {
        k_check_offsets<<<(unsigned)((S + 1 + 255) / 256), 256, 0, st>>>(off, S, n, flagw);
        k_offsets_flag<<<(unsigned)((S + 255) / 256), 256, 0, st>>>(flagw, S, status);
    }
    return status;
}

hipError_t fwd_run(bool boxes, const uint32_t *kind, const float4 *box, int64_t n,
                   const int64_t *off, int64_t S, int32_t *match, int32_t *pm, float4 *out,
                   void *ws, uint32_t *status, hipStream_t st, Variant var) {
    const FwdLayout L = fwd_layout(n, off ? S : 1, sizeof(Box), false);
    char *w = (char *)ws;
    status = prep_status(w, L, off, S, n, status, st, true);
    if (n == 0) return hipGetLastError();
    uint32_t *zst = off ? nullptr : status;
    if (boxes)
        return run_pipeline<true, Box, SinkOut>(kind, box, n, off, S, match, pm, SinkOut{out}, w,
                                                L, status, st, nullptr, var, zst);
    return run_pipeline<false, Box, SinkOut>(kind, box, n, off, S, match, pm, SinkOut{out}, w, L,
                                             status, st, nullptr, var, zst);
}

// ------------------------------------------------- no-allocation variant
// A fixed device array stands in for the caller's workspace, for callers that
// cannot allocate one.  Each GPU holds its own copy for the life of the
// process; every call on a GPU uses that GPU's copy, so calls that overlap on
// one GPU race and must be ordered on one stream.  The pipeline clears the
// only words that must start at zero (status and the offsets flag) itself.
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAXDEV = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAXDEV];  // device address of `scratch`, per device

// The address of the calling device's copy of `scratch`: looked up once per
// device with that device current (the host-side name of the array is only a
// stand-in and must never reach a kernel).
hipError_t scratch_for(hipStream_t st, void **out) {
    int dev = 0;
    hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255u)) return hipErrorInvalidValue;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

hipError_t brackets_run(const uint32_t *tok, int64_t n, int32_t *match, int32_t *pm, void *ws,
                        uint32_t *status, hipStream_t st, Variant var) {
    const FwdLayout L = fwd_layout(n, 1, sizeof(Box), false);
    char *w = (char *)ws;
    status = prep_status(w, L, nullptr, 1, n, status, st, true);
    if (n == 0) return hipGetLastError();
    return run_pipeline<false, Box, SinkOut, true>(tok, nullptr, n, nullptr, 1, match, pm, SinkOut{nullptr},
                                                   w, L, status, st, nullptr, var, status);
}

ComposeF32Layout compose_f32_layout(int64_t n) {
    ComposeF32Layout C{};
    C.f = fwd_layout(n, 1, sizeof(Box), false);
    const int64_t nn = n > 0 ? n : 1;
    size_t o = C.f.total;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    C.pm = take(sizeof(int32_t) * nn);
    C.ptr0 = take(sizeof(int32_t) * nn);
    C.ptr1 = take(sizeof(int32_t) * nn);
    C.val0 = take(24 * (size_t)nn);
    C.val1 = take(24 * (size_t)nn);
    C.flags = take(sizeof(uint32_t) * XJ_ROUNDS);
    C.total = o;
    return C;
}

hipError_t compose_f32_run(const uint32_t *kind, const float *xf, int64_t n, float *out, void *ws,
                           uint32_t *status, hipStream_t st) {
    const ComposeF32Layout C = compose_f32_layout(n);
    char *w = (char *)ws;
    int32_t *pm = (int32_t *)(w + C.pm);
    // the enclosing open of every element: matching's stronger output (Fig. 1)
    hipError_t e = fwd_run(false, kind, nullptr, n, nullptr, 1, nullptr, pm, nullptr, ws, status, st,
                           default_variant(false));
    if (e != hipSuccess || n == 0) return e;
    int32_t *ptr[2] = {(int32_t *)(w + C.ptr0), (int32_t *)(w + C.ptr1)};
    float *val[2] = {(float *)(w + C.val0), (float *)(w + C.val1)};
    uint32_t *flags = (uint32_t *)(w + C.flags);
    int rounds = 0;  // depth < n, so ceil(log2 n) rounds always suffice
    while (((int64_t)1 << rounds) < n) ++rounds;
    const unsigned g = (unsigned)((n + 255) / 256);
    k_zero_status<<<1, XJ_ROUNDS, 0, st>>>(flags, XJ_ROUNDS, flags);
    k_xj_init<<<g, 256, 0, st>>>(kind, xf, pm, n, val[0], ptr[0], flags);
    for (int r = 1; r <= rounds; ++r)
        k_xj_round<<<g, 256, 0, st>>>(r, ptr[(r - 1) & 1], val[(r - 1) & 1], ptr[r & 1], val[r & 1], n,
                                       flags);
    k_xj_out<<<g, 256, 0, st>>>(kind, pm, val[0], val[1], n, out, flags, rounds);
    return hipGetLastError();
}

ReduceUpLayout reduce_up_layout(int64_t n) {
    ReduceUpLayout U{};
    U.f = fwd_layout(n, 1, sizeof(Box), false);
    int64_t N = 1;
    while (N < n) N <<= 1;
    U.N = N;
    size_t o = U.f.total;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    U.match = take(sizeof(int32_t) * (n > 0 ? n : 1));
    U.node = take(24 * (size_t)(2 * N));
    U.total = o;
    return U;
}

hipError_t reduce_up_run(const uint32_t *kind, const float *xf, int64_t n, float *out, void *ws,
                         uint32_t *status, hipStream_t st) {
    const ReduceUpLayout U = reduce_up_layout(n);
    char *w = (char *)ws;
    int32_t *match = (int32_t *)(w + U.match);
    hipError_t e = fwd_run(false, kind, nullptr, n, nullptr, 1, match, nullptr, nullptr, ws, status, st,
                           default_variant(false));
    if (e != hipSuccess || n == 0) return e;
    float *node = (float *)(w + U.node);
    const int64_t N = U.N;
    k_up_leaves<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(kind, xf, n, N, node);
    for (int64_t h = N / 2; h >= 1; h /= 2)
        k_up_level<<<(unsigned)((h + 255) / 256), 256, 0, st>>>(h, node);
    k_up_query<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(kind, xf, match, n, N, node, out);
    return hipGetLastError();
}

hipError_t fwd_run_noalloc(const uint32_t *kind, const float4 *box, int64_t n, int32_t *match,
                           float4 *out, uint32_t *status, hipStream_t st) {
    if (fwd_layout(n, 1, sizeof(Box), false).total > NOALLOC_BYTES) return hipErrorInvalidValue;
    void *ws = nullptr;
    const hipError_t e = scratch_for(st, &ws);
    if (e != hipSuccess) return e;
    return fwd_run(true, kind, box, n, nullptr, 1, match, nullptr, out, ws, status, st,
                   default_variant(true));
}

hipError_t compose_run(const uint32_t *kind, const void *xf, int64_t n, void *out, void *ws,
                       uint32_t *status, hipStream_t st) {
    const FwdLayout L = fwd_layout(n, 1, sizeof(Aff), false);
    char *w = (char *)ws;
    status = prep_status(w, L, nullptr, 1, n, status, st, true);
    if (n == 0) return hipGetLastError();
    return run_pipeline<true, Aff, SinkAff>(kind, (const float4 *)xf, n, nullptr, 1, nullptr, nullptr,
                                            SinkAff{out}, w, L, status, st, nullptr, Variant{}, status);
}

StreamLayout stream_layout(int64_t n) {
    StreamLayout S{};
    S.f = fwd_layout(n, 1, sizeof(Box), false);
    const int64_t nn = n > 0 ? n : 1;
    S.nblk = (nn + CT - 1) / CT;
    size_t o = S.f.total;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    S.ckind = take(sizeof(uint32_t) * nn);
    S.cbox = take(sizeof(float4) * nn);
    S.cidx = take(sizeof(int32_t) * nn);
    S.cmatch = take(sizeof(int32_t) * nn);
    S.cnt = take(sizeof(int) * S.nblk);
    S.m = take(sizeof(int64_t));
    S.total = o;
    return S;
}

hipError_t stream_run(const uint32_t *tag, const float4 *box, int64_t n, int32_t *match,
                      float4 *out, void *ws, uint32_t *status, hipStream_t st) {
    const StreamLayout S = stream_layout(n);
    char *w = (char *)ws;
    status = prep_status(w, S.f, nullptr, 1, n, status, st);
    if (n == 0) return hipGetLastError();
    uint32_t *ckind = (uint32_t *)(w + S.ckind);
    float4 *cbox = (float4 *)(w + S.cbox);
    int32_t *cidx = (int32_t *)(w + S.cidx);
    int32_t *cmatch = (int32_t *)(w + S.cmatch);
    int *cnt = (int *)(w + S.cnt);
    int64_t *m = (int64_t *)(w + S.m);
    k_cmp_count<<<(unsigned)S.nblk, CW, 0, st>>>(tag, n, cnt, status);
    k_cmp_scan<<<1, 1024, 0, st>>>(cnt, S.nblk, m);
    k_cmp_scatter<<<(unsigned)S.nblk, CW, 0, st>>>(tag, box, n, cnt, ckind, cbox, cidx);
    // the pipeline is launched for n elements; partitions past the extracted
    // count m (read on the device) exit at once
    hipError_t e = run_pipeline<true, Box, SinkScatter>(
        ckind, cbox, n, nullptr, 1, match ? cmatch : nullptr, nullptr,
        SinkScatter{out, cidx, (uint32_t)n}, w, S.f, status, st, m);
    if (e != hipSuccess || !match) return e;
    const unsigned g = (unsigned)min((n + 255) / 256, (int64_t)256 * 16);
    k_stream_match<<<g, 256, 0, st>>>(cmatch, cidx, m, match);
    return hipGetLastError();
}

hipError_t bwd_run(const uint32_t *kind, const float4 *box, const float4 *grad_out, int64_t n,
                   float4 *grad_in, void *ws, uint32_t *status, hipStream_t st) {
    const FwdLayout L = fwd_layout(n, 1, sizeof(BoxS), true);
    char *w = (char *)ws;
    status = prep_status(w, L, nullptr, 1, n, status, st, true);
    if (n == 0) return hipGetLastError();
    unsigned long long *acc = (unsigned long long *)(w + L.acc);
    uint8_t *selfm = (uint8_t *)(w + L.selfm);
    k_zero_u64<<<(unsigned)((4 * n + 255) / 256), 256, 0, st>>>(acc, 4 * n);
    hipError_t e = run_pipeline<true, BoxS, SinkGrad>(kind, box, n, nullptr, 1, nullptr, nullptr,
                                                      SinkGrad{grad_out, acc, selfm, n, status}, w, L,
                                                      status, st, nullptr, Variant{}, status);
    if (e != hipSuccess) return e;
    k_grad_final<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(grad_out, acc, selfm, grad_in, n);
    return hipGetLastError();
}

}  // namespace tb
