// Device-side building blocks shared by the libtreebbox kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace tb {

// Partition geometry: one workgroup of W threads handles T = W*K consecutive
// elements; every thread walks K consecutive elements sequentially.
constexpr int WAVE = 64;
constexpr int W = 256;
constexpr int K = 4;
constexpr int T = W * K;
constexpr int NWAVE = W / WAVE;
constexpr int32_t SENT = INT32_MIN;  // "segment reset": below every real level
constexpr int RMAX = 32;             // owner runs stored per partition
constexpr int UB = 256;              // partitions per union block

enum : uint32_t { LEAF = 0, BCLIP = 1, ECLIP = 2, BBLEND = 3, EBLEND = 4 };
enum : uint32_t { ST_BAD_KIND = 1u, ST_UNBAL = 2u, ST_MISMATCH = 4u, ST_BAD_OFF = 8u };
constexpr uint32_t BLEND_BIT = 0x80000000u;  // U-slot index word: open is a blend

__device__ __forceinline__ bool is_open(uint32_t k) { return k == BCLIP || k == BBLEND; }
__device__ __forceinline__ bool is_close(uint32_t k) { return k == ECLIP || k == EBLEND; }

// ------------------------------------------------------------------ boxes
struct Box {
    float x0, y0, x1, y1;
};

__device__ __forceinline__ Box box_inf() { return {-INFINITY, -INFINITY, INFINITY, INFINITY}; }
__device__ __forceinline__ Box box_empty() { return {INFINITY, INFINITY, -INFINITY, -INFINITY}; }
// Intersection and union are exact (max/min never round).
__device__ __forceinline__ Box isect(Box a, Box b) {
    return {fmaxf(a.x0, b.x0), fmaxf(a.y0, b.y0), fminf(a.x1, b.x1), fminf(a.y1, b.y1)};
}
__device__ __forceinline__ Box unite(Box a, Box b) {
    return {fminf(a.x0, b.x0), fminf(a.y0, b.y0), fmaxf(a.x1, b.x1), fmaxf(a.y1, b.y1)};
}
__device__ __forceinline__ Box canon(Box a) {
    return (a.x0 < a.x1 && a.y0 < a.y1) ? a : box_empty();
}
__device__ __forceinline__ Box ld_box(const float4 *p, int64_t i) {
    float4 v = p[i];
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void st_box(float4 *p, int64_t i, Box b) {
    p[i] = make_float4(b.x0, b.y0, b.x1, b.y1);
}

// Box with, per coordinate, the index of the input element attaining it
// (the gradient's route), held as one 64-bit key per coordinate: the
// value's order-preserving bits above 32 bits of index.  The minimum
// coordinates (x0, y0) carry the index and the maximum coordinates (x1, y1)
// its complement, so a union (a plain 64-bit min of x0, y0 and max of x1,
// y1) takes the extreme value and, on equal values, the lower index; an
// intersection flips the index bits around the same compare.  On equal
// values the lower index always wins, so the combine stays associative,
// commutative and idempotent and every combine order yields the same route.
// -0 orders as +0, as the float comparison has them equal.
struct BoxS {
    uint64_t k0, k1, k2, k3;
};
constexpr int32_t NOSRC = INT32_MAX;  // identity elements route nowhere
constexpr uint64_t KLOW = 0xFFFFFFFFull;

__device__ __forceinline__ uint32_t ordf(float f) {
    const uint32_t b = __float_as_uint(f == 0.0f ? 0.0f : f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ uint64_t fkey(float f, uint32_t low) { return ((uint64_t)ordf(f) << 32) | low; }
__device__ __forceinline__ uint64_t kmin(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t kmax(uint64_t a, uint64_t b) { return a > b ? a : b; }
// the larger value, the lower index on a tie (key holding the index)
__device__ __forceinline__ uint64_t kmax_lo(uint64_t a, uint64_t b) { return (a ^ KLOW) > (b ^ KLOW) ? a : b; }
// the smaller value, the lower index on a tie (key holding the complement)
__device__ __forceinline__ uint64_t kmin_lo(uint64_t a, uint64_t b) { return (a ^ KLOW) < (b ^ KLOW) ? a : b; }
__device__ __forceinline__ BoxS isect(const BoxS &a, const BoxS &b) {
    return {kmax_lo(a.k0, b.k0), kmax_lo(a.k1, b.k1), kmin_lo(a.k2, b.k2), kmin_lo(a.k3, b.k3)};
}
__device__ __forceinline__ BoxS unite(const BoxS &a, const BoxS &b) {
    return {kmin(a.k0, b.k0), kmin(a.k1, b.k1), kmax(a.k2, b.k2), kmax(a.k3, b.k3)};
}
__device__ __forceinline__ bool boxs_nonempty(const BoxS &a) {
    return (uint32_t)(a.k0 >> 32) < (uint32_t)(a.k2 >> 32) && (uint32_t)(a.k1 >> 32) < (uint32_t)(a.k3 >> 32);
}
__device__ __forceinline__ BoxS boxs_empty() {
    return {fkey(INFINITY, NOSRC), fkey(INFINITY, NOSRC), fkey(-INFINITY, ~(uint32_t)NOSRC),
            fkey(-INFINITY, ~(uint32_t)NOSRC)};
}
__device__ __forceinline__ BoxS canon(const BoxS &a) {
    const bool ne = boxs_nonempty(a);
    const BoxS e = boxs_empty();
    return {ne ? a.k0 : e.k0, ne ? a.k1 : e.k1, ne ? a.k2 : e.k2, ne ? a.k3 : e.k3};
}
// the attaining element of coordinate c (NOSRC for none)
__device__ __forceinline__ int32_t boxs_src(const BoxS &a, int c) {
    return c == 0 ? (int32_t)(uint32_t)a.k0
         : c == 1 ? (int32_t)(uint32_t)a.k1
         : c == 2 ? (int32_t)~(uint32_t)a.k2
                  : (int32_t)~(uint32_t)a.k3;
}

template <class V>
__device__ __forceinline__ V vsel(bool c, const V &a, const V &b) {
    return c ? a : b;
}
// Component-wise select.  A conditional expression on two payload lvalues
// is a select of their addresses, which can keep the payloads in scratch
// memory; this builds the result from selected scalars instead.
__device__ __forceinline__ Box vsel(bool c, const Box &a, const Box &b) {
    return {c ? a.x0 : b.x0, c ? a.y0 : b.y0, c ? a.x1 : b.x1, c ? a.y1 : b.y1};
}
__device__ __forceinline__ BoxS vsel(bool c, const BoxS &a, const BoxS &b) {
    return {c ? a.k0 : b.k0, c ? a.k1 : b.k1, c ? a.k2 : b.k2, c ? a.k3 : b.k3};
}

// Payload traits: identities, own element, workspace load/store.
template <class V>
struct Pay;
template <>
struct Pay<Box> {
    static __device__ __forceinline__ Box inf() { return box_inf(); }
    static __device__ __forceinline__ Box empty() { return box_empty(); }
    static constexpr bool kUnions = true;     // blend unions up the tree
    static constexpr bool kLeafOwn = true;    // a leaf's row combines its own input
    static constexpr bool kAllOpens = false;  // both open kinds carry a payload
    static __device__ __forceinline__ Box own(float4 b, int64_t) { return {b.x, b.y, b.z, b.w}; }
    static __device__ __forceinline__ Box in(const void *base, int64_t i) {
        return own(((const float4 *)base)[i], i);
    }
    static __device__ __forceinline__ Box ld(const void *base, int64_t i) {
        return ld_box((const float4 *)base, i);
    }
    static __device__ __forceinline__ void st(void *base, int64_t i, Box v) {
        st_box((float4 *)base, i, v);
    }
    static __device__ __forceinline__ bool nonempty(const Box &v) { return v.x0 < v.x1 && v.y0 < v.y1; }
};
template <>
struct Pay<BoxS> {
    static __device__ __forceinline__ BoxS inf() {
        return {fkey(-INFINITY, NOSRC), fkey(-INFINITY, NOSRC), fkey(INFINITY, ~(uint32_t)NOSRC),
                fkey(INFINITY, ~(uint32_t)NOSRC)};
    }
    static __device__ __forceinline__ BoxS empty() { return boxs_empty(); }
    static constexpr bool kUnions = true;
    static constexpr bool kLeafOwn = true;
    static constexpr bool kAllOpens = false;
    static __device__ __forceinline__ BoxS in(const void *base, int64_t i) {
        return own(((const float4 *)base)[i], i);
    }
    static __device__ __forceinline__ BoxS own(float4 b, int64_t i) {
        const uint32_t s = (uint32_t)i;
        return {fkey(b.x, s), fkey(b.y, s), fkey(b.z, ~s), fkey(b.w, ~s)};
    }
    // rows of 32 bytes: two 16-byte halves
    static __device__ __forceinline__ BoxS ld(const void *base, int64_t i) {
        const ulonglong2 a = ((const ulonglong2 *)base)[2 * i];
        const ulonglong2 b = ((const ulonglong2 *)base)[2 * i + 1];
        return {a.x, a.y, b.x, b.y};
    }
    static __device__ __forceinline__ void st(void *base, int64_t i, const BoxS &v) {
        ulonglong2 a, b;
        a.x = v.k0, a.y = v.k1, b.x = v.k2, b.y = v.k3;
        ((ulonglong2 *)base)[2 * i] = a;
        ((ulonglong2 *)base)[2 * i + 1] = b;
    }
    static __device__ __forceinline__ bool nonempty(const BoxS &v) { return boxs_nonempty(v); }
};

// A 2-D affine transform [a b c; d e f] on integer coordinates, arithmetic
// modulo 2^32: exact, hence associative, and not commutative.  As a payload
// composed down the tree, "isect(p, q)" is p . q (q applied first): the
// enclosing transform p always comes first at every combine.
struct Aff {
    uint32_t a, b, c, d, e, f;
};
__device__ __forceinline__ Aff aff_id() { return {1u, 0u, 0u, 0u, 1u, 0u}; }
__device__ __forceinline__ Aff isect(const Aff &p, const Aff &q) {
    return {p.a * q.a + p.b * q.d, p.a * q.b + p.b * q.e, p.a * q.c + p.b * q.f + p.c,
            p.d * q.a + p.e * q.d, p.d * q.b + p.e * q.e, p.d * q.c + p.e * q.f + p.f};
}
// there is nothing to combine upwards; the union steps are compiled out
__device__ __forceinline__ Aff unite(Aff a, const Aff &) { return a; }
__device__ __forceinline__ Aff canon(Aff a) { return a; }
__device__ __forceinline__ Aff vsel(bool c, const Aff &a, const Aff &b) {
    return {c ? a.a : b.a, c ? a.b : b.b, c ? a.c : b.c, c ? a.d : b.d, c ? a.e : b.e, c ? a.f : b.f};
}
template <>
struct Pay<Aff> {
    static constexpr bool kUnions = false;
    static constexpr bool kLeafOwn = false;
    static constexpr bool kAllOpens = true;
    static __device__ __forceinline__ Aff inf() { return aff_id(); }
    static __device__ __forceinline__ Aff empty() { return aff_id(); }
    // rows of 24 bytes, 8-byte aligned
    static __device__ __forceinline__ Aff ld(const void *base, int64_t i) {
        const uint2 *q = (const uint2 *)base + 3 * i;
        const uint2 x = q[0], y = q[1], z = q[2];
        return {x.x, x.y, y.x, y.y, z.x, z.y};
    }
    static __device__ __forceinline__ Aff in(const void *base, int64_t i) { return ld(base, i); }
    static __device__ __forceinline__ void st(void *base, int64_t i, const Aff &v) {
        uint2 *q = (uint2 *)base + 3 * i;
        q[0] = make_uint2(v.a, v.b);
        q[1] = make_uint2(v.c, v.d);
        q[2] = make_uint2(v.e, v.f);
    }
    static __device__ __forceinline__ bool nonempty(const Aff &) { return true; }
};

// ---------------------------------------------------------- wave shuffles
// DPP lane moves (GFX9 data-parallel primitives): the source lane is read
// through the VALU crossbar, with no LDS round trip.  Lanes whose source lies
// outside the pattern, or outside `RM` (a mask of 16-lane rows), keep `old`.
namespace dpp {
constexpr int SHR1 = 0x111, SHR2 = 0x112, SHR4 = 0x114, SHR8 = 0x118;  // lane i <- i-k, in row
constexpr int SHL1 = 0x101, SHL2 = 0x102, SHL4 = 0x104, SHL8 = 0x108;  // lane i <- i+k, in row
constexpr int WSHR1 = 0x138, WSHL1 = 0x130;                            // lane i <- i-1 / i+1
constexpr int BC15 = 0x142, BC31 = 0x143;  // row r <- lane 16r-1 / lane 31
}  // namespace dpp
template <int C, int RM = 0xF>
__device__ __forceinline__ int dmov(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, C, RM, 0xF, false);
}
template <int C, int RM = 0xF>
__device__ __forceinline__ float dmov(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), C, RM, 0xF, false));
}
template <int C, int RM = 0xF>
__device__ __forceinline__ Box dmov(Box o, Box v) {
    return {dmov<C, RM>(o.x0, v.x0), dmov<C, RM>(o.y0, v.y0), dmov<C, RM>(o.x1, v.x1), dmov<C, RM>(o.y1, v.y1)};
}
template <int C, int RM = 0xF>
__device__ __forceinline__ uint64_t dmov64(uint64_t o, uint64_t v) {
    const uint32_t lo = (uint32_t)dmov<C, RM>((int)(uint32_t)o, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)dmov<C, RM>((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <int C, int RM = 0xF>
__device__ __forceinline__ BoxS dmov(BoxS o, BoxS v) {
    return {dmov64<C, RM>(o.k0, v.k0), dmov64<C, RM>(o.k1, v.k1), dmov64<C, RM>(o.k2, v.k2), dmov64<C, RM>(o.k3, v.k3)};
}
// uniform read of one lane
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ Box rdlane(Box v, int l) {
    return {rdlane(v.x0, l), rdlane(v.y0, l), rdlane(v.x1, l), rdlane(v.y1, l)};
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
    const uint32_t lo = (uint32_t)rdlane((int)(uint32_t)v, l), hi = (uint32_t)rdlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ BoxS rdlane(BoxS v, int l) {
    return {rdlane64(v.k0, l), rdlane64(v.k1, l), rdlane64(v.k2, l), rdlane64(v.k3, l)};
}

template <int C, int RM = 0xF>
__device__ __forceinline__ Aff dmov(Aff o, Aff v) {
    return {(uint32_t)dmov<C, RM>((int)o.a, (int)v.a), (uint32_t)dmov<C, RM>((int)o.b, (int)v.b),
            (uint32_t)dmov<C, RM>((int)o.c, (int)v.c), (uint32_t)dmov<C, RM>((int)o.d, (int)v.d),
            (uint32_t)dmov<C, RM>((int)o.e, (int)v.e), (uint32_t)dmov<C, RM>((int)o.f, (int)v.f)};
}
__device__ __forceinline__ Aff rdlane(Aff v, int l) {
    return {(uint32_t)rdlane((int)v.a, l), (uint32_t)rdlane((int)v.b, l), (uint32_t)rdlane((int)v.c, l),
            (uint32_t)rdlane((int)v.d, l), (uint32_t)rdlane((int)v.e, l), (uint32_t)rdlane((int)v.f, l)};
}
__device__ __forceinline__ Aff shfl_idx(Aff v, int src) {
    return {(uint32_t)__shfl((int)v.a, src, WAVE), (uint32_t)__shfl((int)v.b, src, WAVE),
            (uint32_t)__shfl((int)v.c, src, WAVE), (uint32_t)__shfl((int)v.d, src, WAVE),
            (uint32_t)__shfl((int)v.e, src, WAVE), (uint32_t)__shfl((int)v.f, src, WAVE)};
}
// arbitrary-lane reads
__device__ __forceinline__ Box shfl_idx(Box v, int src) {
    return {__shfl(v.x0, src, WAVE), __shfl(v.y0, src, WAVE), __shfl(v.x1, src, WAVE), __shfl(v.y1, src, WAVE)};
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, WAVE);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, WAVE);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ BoxS shfl_idx(BoxS v, int src) {
    return {shfl64(v.k0, src), shfl64(v.k1, src), shfl64(v.k2, src), shfl64(v.k3, src)};
}

// Segmented sum: (r, v) with r = "a reset occurs in this range"; a reset
// discards everything to its left.
struct Seg {
    int r, v;
};
template <int C, int RM = 0xF>
__device__ __forceinline__ Seg dmov(Seg o, Seg v) { return {dmov<C, RM>(o.r, v.r), dmov<C, RM>(o.v, v.v)}; }
__device__ __forceinline__ Seg rdlane(Seg v, int l) { return {rdlane(v.r, l), rdlane(v.v, l)}; }
struct SegOp {
    __device__ Seg operator()(Seg x, Seg y) const { return y.r ? y : Seg{x.r, x.v + y.v}; }
};
// A segmented sum carried together with a plain sum u.
struct SegU {
    int r, v, u;
};
template <int C, int RM = 0xF>
__device__ __forceinline__ SegU dmov(SegU o, SegU v) {
    return {dmov<C, RM>(o.r, v.r), dmov<C, RM>(o.v, v.v), dmov<C, RM>(o.u, v.u)};
}
__device__ __forceinline__ SegU rdlane(SegU v, int l) { return {rdlane(v.r, l), rdlane(v.v, l), rdlane(v.u, l)}; }
struct SegUOp {
    __device__ SegU operator()(SegU x, SegU y) const {
        return y.r ? SegU{1, y.v, x.u + y.u} : SegU{x.r, x.v + y.v, x.u + y.u};
    }
};
// Bicyclic element with scene resets: (a pops of the stack below, b
// unmatched opens left, r a reset occurred).  (a,b) ⊕ (c,d) is the paper's
// bicyclic product; a reset clears what lies to its left, so pops after it
// never reach further down.
struct BicR {
    int a, b, r;
};
template <int C, int RM = 0xF>
__device__ __forceinline__ BicR dmov(BicR o, BicR v) {
    return {dmov<C, RM>(o.a, v.a), dmov<C, RM>(o.b, v.b), dmov<C, RM>(o.r, v.r)};
}
__device__ __forceinline__ BicR rdlane(BicR v, int l) { return {rdlane(v.a, l), rdlane(v.b, l), rdlane(v.r, l)}; }
__device__ __forceinline__ BicR bicr(const BicR &x, const BicR &y) {
    const int m = x.b < y.a ? x.b : y.a;
    return {x.a + (x.r ? 0 : y.a - m), y.r ? y.b : x.b + y.b - m, x.r | y.r};
}
struct BicROp {
    __device__ BicR operator()(BicR x, BicR y) const { return bicr(x, y); }
};
struct MinOp {
    __device__ int operator()(int a, int b) const { return a < b ? a : b; }
};
struct AddOp {
    __device__ int operator()(int a, int b) const { return a + b; }
};
struct IsectOp {
    template <class V>
    __device__ V operator()(V a, V b) const { return isect(a, b); }
};
struct UniteOp {
    template <class V>
    __device__ V operator()(V a, V b) const { return unite(a, b); }
};

__device__ __forceinline__ BicR shfl_idx(BicR x, int src) {
    return {__shfl(x.a, src, WAVE), __shfl(x.b, src, WAVE), __shfl(x.r, src, WAVE)};
}
__device__ __forceinline__ int shfl_idx(int x, int src) { return __shfl(x, src, WAVE); }

// Box min/max steps as DPP-modified VALU ops: each component is combined
// with its DPP source lane in one instruction (the compiler forms this only
// for integer ops).  Lanes without a source keep their value, which is the
// identity behaviour for these idempotent combines.  The leading s_nop covers
// the wait states a DPP read needs after a VALU write of its source or of
// EXEC; inside a block every component is written three instructions before
// its next DPP read.
#define TB_DPP4(OA, OB, CTRL)                                                                          \
    OA " %0, %0, %0 " CTRL "\n\t" OA " %1, %1, %1 " CTRL "\n\t" OB " %2, %2, %2 " CTRL "\n\t" OB \
       " %3, %3, %3 " CTRL "\n\t"
#define TB_DPP_UNITE(CTRL) TB_DPP4("v_min_f32_dpp", "v_max_f32_dpp", CTRL)
#define TB_DPP_ISECT(CTRL) TB_DPP4("v_max_f32_dpp", "v_min_f32_dpp", CTRL)
#define TB_BOX_OPS(b) "+v"(b.x0), "+v"(b.y0), "+v"(b.x1), "+v"(b.y1)
// one scan step (row_shr 1, 2, 4, 8, then row_bcast 15 and 31), unite
template <int STEP>
__device__ __forceinline__ void box_unite_step(Box &b) {
    if constexpr (STEP == 0) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shr:1 row_mask:0xf bank_mask:0xf") : TB_BOX_OPS(b));
    if constexpr (STEP == 1) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shr:2 row_mask:0xf bank_mask:0xf") : TB_BOX_OPS(b));
    if constexpr (STEP == 2) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shr:4 row_mask:0xf bank_mask:0xf") : TB_BOX_OPS(b));
    if constexpr (STEP == 3) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shr:8 row_mask:0xf bank_mask:0xf") : TB_BOX_OPS(b));
    if constexpr (STEP == 4) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_bcast:15 row_mask:0xa bank_mask:0xf") : TB_BOX_OPS(b));
    if constexpr (STEP == 5) asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_bcast:31 row_mask:0xc bank_mask:0xf") : TB_BOX_OPS(b));
}
// the six steps of an inclusive wave scan in one block
template <bool UNITE>
__device__ __forceinline__ void box_incl_scan_dpp(Box &b) {
    if constexpr (UNITE)
        asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shr:1 row_mask:0xf bank_mask:0xf")
                         TB_DPP_UNITE("row_shr:2 row_mask:0xf bank_mask:0xf")
                             TB_DPP_UNITE("row_shr:4 row_mask:0xf bank_mask:0xf")
                                 TB_DPP_UNITE("row_shr:8 row_mask:0xf bank_mask:0xf")
                                     TB_DPP_UNITE("row_bcast:15 row_mask:0xa bank_mask:0xf")
                                         TB_DPP_UNITE("row_bcast:31 row_mask:0xc bank_mask:0xf") "s_nop 1"
                     : TB_BOX_OPS(b));
    else
        asm volatile("s_nop 4\n\t" TB_DPP_ISECT("row_shr:1 row_mask:0xf bank_mask:0xf")
                         TB_DPP_ISECT("row_shr:2 row_mask:0xf bank_mask:0xf")
                             TB_DPP_ISECT("row_shr:4 row_mask:0xf bank_mask:0xf")
                                 TB_DPP_ISECT("row_shr:8 row_mask:0xf bank_mask:0xf")
                                     TB_DPP_ISECT("row_bcast:15 row_mask:0xa bank_mask:0xf")
                                         TB_DPP_ISECT("row_bcast:31 row_mask:0xc bank_mask:0xf") "s_nop 1"
                     : TB_BOX_OPS(b));
}
// in-row suffix steps (lane i combines lane i + 1, 2, 4, 8 of its row)
template <bool UNITE>
__device__ __forceinline__ void box_suffix_rows_dpp(Box &b) {
    if constexpr (UNITE)
        asm volatile("s_nop 4\n\t" TB_DPP_UNITE("row_shl:1 row_mask:0xf bank_mask:0xf")
                         TB_DPP_UNITE("row_shl:2 row_mask:0xf bank_mask:0xf")
                             TB_DPP_UNITE("row_shl:4 row_mask:0xf bank_mask:0xf")
                                 TB_DPP_UNITE("row_shl:8 row_mask:0xf bank_mask:0xf") "s_nop 1"
                     : TB_BOX_OPS(b));
    else
        asm volatile("s_nop 4\n\t" TB_DPP_ISECT("row_shl:1 row_mask:0xf bank_mask:0xf")
                         TB_DPP_ISECT("row_shl:2 row_mask:0xf bank_mask:0xf")
                             TB_DPP_ISECT("row_shl:4 row_mask:0xf bank_mask:0xf")
                                 TB_DPP_ISECT("row_shl:8 row_mask:0xf bank_mask:0xf") "s_nop 1"
                     : TB_BOX_OPS(b));
}
template <class V, class Op>
constexpr bool kBoxDpp = std::is_same<V, Box>::value && (std::is_same<Op, UniteOp>::value || std::is_same<Op, IsectOp>::value);

// Inclusive scan inside one wave for an associative `op` with identity `id`
// (operands in lane order): in-row steps of 1, 2, 4, 8 lanes, then the row
// totals are carried across rows 0->1, 2->3 and 1->2,3.
template <class V, class Op>
__device__ __forceinline__ V wave_incl_scan(V v, Op op, V id) {
    if constexpr (kBoxDpp<V, Op>) {
        box_incl_scan_dpp<std::is_same<Op, UniteOp>::value>(v);
        return v;
    }
    v = op(dmov<dpp::SHR1>(id, v), v);
    v = op(dmov<dpp::SHR2>(id, v), v);
    v = op(dmov<dpp::SHR4>(id, v), v);
    v = op(dmov<dpp::SHR8>(id, v), v);
    v = op(dmov<dpp::BC15, 0xA>(id, v), v);
    v = op(dmov<dpp::BC31, 0xC>(id, v), v);
    return v;
}

// Exclusive scan inside one wave; also returns the wave total.
template <class V, class Op>
__device__ __forceinline__ V wave_excl_scan(V v, Op op, V ident, V *total) {
    const V inc = wave_incl_scan(v, op, ident);
    *total = rdlane(inc, WAVE - 1);
    return dmov<dpp::WSHR1>(ident, inc);
}

// Exclusive suffix scan inside one wave: lane l gets op over lanes l+1..63
// in lane order (identity at lane 63); also returns the wave total.
template <class V, class Op>
__device__ __forceinline__ V wave_excl_suffix_scan(V v, Op op, V id, V *total) {
    if constexpr (kBoxDpp<V, Op>) {
        box_suffix_rows_dpp<std::is_same<Op, UniteOp>::value>(v);
    } else {
        v = op(v, dmov<dpp::SHL1>(id, v));
        v = op(v, dmov<dpp::SHL2>(id, v));
        v = op(v, dmov<dpp::SHL4>(id, v));
        v = op(v, dmov<dpp::SHL8>(id, v));
    }
    // lanes 16r hold row r's suffix; carry the later rows' product in
    const V t1 = rdlane(v, 16), t2 = rdlane(v, 32), t3 = rdlane(v, 48);
    const V r1 = op(t2, t3), r0 = op(t1, r1);
    const int row = (threadIdx.x & (WAVE - 1)) >> 4;
    const V later = vsel(row == 0, r0, vsel(row == 1, r1, vsel(row == 2, t3, id)));
    v = op(v, later);
    *total = rdlane(v, 0);
    return dmov<dpp::WSHL1>(id, v);
}

// Exclusive scan over the NW*64 threads of a workgroup; `sh` holds NW values.
// Also returns the workgroup total.  Contains two barriers (one when `sh` is
// not used again, REUSE = false).
template <int NW, class V, class Op, bool REUSE = true>
__device__ __forceinline__ V block_excl_scan(V v, Op op, V ident, V *sh, V *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    V inc = wave_incl_scan(v, op, ident);
    if (lane == WAVE - 1) sh[wid] = inc;
    __syncthreads();
    V pre = ident, tot = ident;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w < wid) pre = op(pre, sh[w]);
        tot = op(tot, sh[w]);
    }
    const V ex = dmov<dpp::WSHR1>(ident, inc);
    *total = tot;
    if (REUSE) __syncthreads();  // `sh` may be written again after return
    return op(pre, ex);
}

// Typed bracket tokens: 0 is no bracket, 2t+1 opens type t, 2t+2 closes it;
// the structure alone, as kinds
__device__ __forceinline__ uint32_t bracket_kind(uint32_t tok) {
    return tok == 0u ? (uint32_t)LEAF : (tok & 1u) ? (uint32_t)BCLIP : (uint32_t)ECLIP;
}

// both open kinds as BEGIN_CLIP and both closes as END_CLIP (payloads that
// every open carries)
__device__ __forceinline__ uint32_t as_clip(uint32_t k) {
    return k == BBLEND ? (uint32_t)BCLIP : k == EBLEND ? (uint32_t)ECLIP : k;
}

// ----------------------------------------------------------- small helpers
__device__ __forceinline__ int msb32(uint32_t x) { return 31 - __clz(x); }

// lower_bound over off[0..cnt): first index with off[idx] >= x
__device__ __forceinline__ int64_t lower_bound64(const int64_t *off, int64_t cnt, int64_t x) {
    int64_t lo = 0, hi = cnt;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// scene holding element i: last s with off[s] <= i, clamped to [0, S-1]
__device__ __forceinline__ int64_t scene_of(const int64_t *off, int64_t S, int64_t i) {
    if (!off) return 0;
    int64_t lo = 0, hi = S + 1;  // first index with off[idx] > i
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid + 1;
        else
            hi = mid;
    }
    int64_t s = lo - 1;
    return s < 0 ? 0 : (s >= S ? S - 1 : s);
}

// Scene starts inside [g0, g0+KK) as a bit mask (bit j: element g0+j starts a
// scene).  Without offsets the only start is element 0.  Only o[0..S-1] are
// scene starts, and only those below n: the end sentinel o[S] = n (and the
// start of an empty scene at the end) is no element, so it resets nothing.
template <int KK = K>
__device__ __forceinline__ uint32_t reset_mask(const int64_t *off, int64_t S, int64_t n, int64_t g0) {
    if (!off) return g0 == 0 ? 1u : 0u;
    uint32_t r = 0;
    for (int64_t s = lower_bound64(off, S, g0); s < S; ++s) {
        int64_t o = off[s];
        if (o >= g0 + KK || o >= n) break;
        if (o >= g0) r |= 1u << (o - g0);
    }
    return r;
}

__device__ __forceinline__ void flag(uint32_t *status, const int64_t *off, int64_t S, int64_t i,
                                     uint32_t bits) {
    atomicOr(status + scene_of(off, S, i), bits);
}

// Loads KK kinds of one thread; elements at or past n read as LEAF.
template <int KK>
__device__ __forceinline__ void load_kinds(const uint32_t *kind, int64_t n, int64_t g0,
                                           uint32_t (&ks)[KK]) {
    static_assert(KK % 4 == 0, "kinds load in groups of four");
    // 16-byte loads need a 16-byte aligned array (the caller's may be 4)
    if (g0 + KK <= n && ((uintptr_t)kind & 15u) == 0) {
#pragma unroll
        for (int q = 0; q < KK / 4; ++q) {
            const uint4 v = *reinterpret_cast<const uint4 *>(kind + g0 + 4 * q);
            ks[4 * q] = v.x, ks[4 * q + 1] = v.y, ks[4 * q + 2] = v.z, ks[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < KK; ++j) ks[j] = (g0 + j < n) ? kind[g0 + j] : LEAF;
    }
}

// Per-thread sequential walk over K kinds with a bitmask stack of local
// opens (the top is the highest set bit).  Returns the pops of the incoming
// stack before the first scene start (a), the mask of unmatched opens after
// the last scene start, and whether a scene starts in this thread.
struct Walk {
    int a;
    uint32_t umask;
    bool rs;
};
template <int KK>
__device__ __forceinline__ Walk walk_kinds(const uint32_t (&ks)[KK], uint32_t rm) {
    uint32_t mask = 0;
    int a = 0;
    bool rs = false;
#pragma unroll
    for (int j = 0; j < KK; ++j) {
        if ((rm >> j) & 1u) {
            mask = 0;
            rs = true;
        }
        uint32_t k = ks[j];
        if (is_open(k))
            mask |= 1u << j;
        else if (is_close(k)) {
            if (mask)
                mask &= ~(1u << msb32(mask));
            else if (!rs)
                ++a;
        }
    }
    return {a, mask, rs};
}

// ------------------------------------------------ LDS min tree over WW ints
// mt[WW + i] = leaf i; mt[x] = min(mt[2x], mt[2x+1]) for WW/64 <= x < WW
// (down to one node per wave; see mintree_node for the nodes above).
// Thread t supplies leaf t.  The levels are formed with DPP row shifts and
// broadcasts inside each wave.  One barrier.
template <int WW = W>
__device__ __forceinline__ void mintree_build(int *mt, int v) {
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    mt[WW + t] = v;
    // after step l, a lane whose low l bits are all set holds the min of its
    // aligned group of 2^l lanes (out-of-pattern lanes combine with themselves)
    v = min(v, dmov<dpp::SHR1>(INT32_MAX, v));
    if ((lane & 1) == 1) mt[(WW + t) >> 1] = v;
    v = min(v, dmov<dpp::SHR2>(INT32_MAX, v));
    if ((lane & 3) == 3) mt[(WW + t) >> 2] = v;
    v = min(v, dmov<dpp::SHR4>(INT32_MAX, v));
    if ((lane & 7) == 7) mt[(WW + t) >> 3] = v;
    v = min(v, dmov<dpp::SHR8>(INT32_MAX, v));
    if ((lane & 15) == 15) mt[(WW + t) >> 4] = v;
    v = min(v, dmov<dpp::BC15, 0xA>(INT32_MAX, v));
    if ((lane & 31) == 31) mt[(WW + t) >> 5] = v;
    v = min(v, dmov<dpp::BC31, 0xC>(INT32_MAX, v));
    if (lane == 63) mt[(WW + t) >> 6] = v;
    __syncthreads();
}

// A min-tree node; nodes above the wave level (index < WW/64) are not
// stored and come from the wave nodes below them.
template <int WW = W>
__device__ __forceinline__ int mintree_node(const int *mt, int x) {
    constexpr int NW = WW / WAVE;
    static_assert(NW == 1 || NW == 2 || NW == 4, "one, two or four waves");
    if (x >= NW) return mt[x];
    if (NW == 2) return min(mt[2], mt[3]);  // x == 1
    if (x == 2) return min(mt[4], mt[5]);
    if (x == 3) return min(mt[6], mt[7]);
    return min(min(mt[4], mt[5]), min(mt[6], mt[7]));
}

// The wave levels of a union tree over the WW threads (leaves at WW + t,
// internal nodes down to one node per wave, i.e. indices WW/64..WW/32-1,
// and EMPTY at index 0; nodes above the wave level are not built) and the
// wave's exclusive prefix union, in one pass: after each inclusive-scan step
// the lanes that close an aligned group of 2, 4, ... 64 lanes hold that
// group's union, which is the tree node.  No barrier.
template <class V, int WW>
__device__ __forceinline__ V uniontree_scan(V *ut, V v, V *total) {
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    if (t == 0) ut[0] = Pay<V>::empty();
    ut[WW + t] = v;
    if constexpr (std::is_same<V, Box>::value) {
        box_unite_step<0>(v);
        if ((lane & 1) == 1) ut[(WW + t) >> 1] = v;
        box_unite_step<1>(v);
        if ((lane & 3) == 3) ut[(WW + t) >> 2] = v;
        box_unite_step<2>(v);
        if ((lane & 7) == 7) ut[(WW + t) >> 3] = v;
        box_unite_step<3>(v);
        if ((lane & 15) == 15) ut[(WW + t) >> 4] = v;
        box_unite_step<4>(v);
        if ((lane & 31) == 31) ut[(WW + t) >> 5] = v;
        box_unite_step<5>(v);
        if (lane == 63) ut[(WW + t) >> 6] = v;
        asm volatile("s_nop 1" ::: "memory");
    } else {
        v = unite(v, dmov<dpp::SHR1>(v, v));
        if ((lane & 1) == 1) ut[(WW + t) >> 1] = v;
        v = unite(v, dmov<dpp::SHR2>(v, v));
        if ((lane & 3) == 3) ut[(WW + t) >> 2] = v;
        v = unite(v, dmov<dpp::SHR4>(v, v));
        if ((lane & 7) == 7) ut[(WW + t) >> 3] = v;
        v = unite(v, dmov<dpp::SHR8>(v, v));
        if ((lane & 15) == 15) ut[(WW + t) >> 4] = v;
        v = unite(v, dmov<dpp::BC15, 0xA>(v, v));
        if ((lane & 31) == 31) ut[(WW + t) >> 5] = v;
        v = unite(v, dmov<dpp::BC31, 0xC>(v, v));
        if (lane == 63) ut[(WW + t) >> 6] = v;
    }
    *total = rdlane(v, WAVE - 1);
    return dmov<dpp::WSHR1>(Pay<V>::empty(), v);
}

// Rightmost leaf s < t with leaf value < v, or -1.  The left siblings of
// every ancestor of leaf t are read together (the lowest one below v holds
// the answer), then the descent takes two levels per step, reading three
// grandchildren at once.  Every read is unconditional (nodes above the wave
// level come from the wave nodes), so the reads of a step are in flight
// together rather than one dependent read per level.
template <int WW = W>
__device__ __forceinline__ int mintree_prev_less(const int *mt, int t, int v) {
    constexpr int NW = WW / WAVE;
    static_assert(NW == 1 || NW == 2 || NW == 4, "one, two or four waves");
    constexpr int LV = NW == 4 ? 8 : NW == 2 ? 7 : 6;  // levels below the root
    // nodes 1 .. NW-1 (not stored)
    int up1 = INT32_MAX, up2 = INT32_MAX, up3 = INT32_MAX;
    if (NW == 4) {
        const int4 wn = *reinterpret_cast<const int4 *>(mt + 4);
        up2 = min(wn.x, wn.y), up3 = min(wn.z, wn.w), up1 = min(up2, up3);
    }
    const int x = WW + t;
    int y = 0, lev = 0;
    int cv[LV];
#pragma unroll
    for (int k = 0; k < LV; ++k) {
        const int c = (x >> k) - 1;  // the left sibling when x >> k is a right child
        const int m = mt[c >= NW ? c : NW];
        cv[k] = !((x >> k) & 1) ? INT32_MAX : c >= NW ? m : c == 3 ? up3 : c == 2 ? up2 : up1;
    }
#pragma unroll
    for (int k = LV - 1; k >= 0; --k)
        if (cv[k] < v) y = (x >> k) - 1, lev = k;
    if (y == 0) return -1;
    while (lev >= 2) {
        const int a3 = mt[4 * y + 3], a2 = mt[4 * y + 2], a1 = mt[4 * y + 1];
        y = a3 < v ? 4 * y + 3 : a2 < v ? 4 * y + 2 : a1 < v ? 4 * y + 1 : 4 * y;
        lev -= 2;
    }
    if (lev == 1) y = mt[2 * y + 1] < v ? 2 * y + 1 : 2 * y;
    return y - WW;
}

// Union over leaves [lo, hi] of a tree built by uniontree_scan, for
// 1 <= lo and hi <= WW-2 (EMPTY if lo > hi).  Such a range never covers a
// node above the wave level (at most four waves), so seven levels suffice.
// Straight-line: every LDS read is issued before the first is used; a level
// that contributes nothing reads node 0, which uniontree_scan sets to EMPTY.
template <class V, int WW = W>
__device__ __forceinline__ V uniontree_inner(const V *ut, int lo, int hi) {
    static_assert(WW / WAVE <= 4, "ranges inside at most four waves");
    // Level k of the half-open range [l, h) is [ceil(l / 2^k), floor(h / 2^k)):
    // its odd left end and its odd right end are the nodes taken there.
    V r = Pay<V>::empty();
    const uint32_t l = (uint32_t)(lo + WW), h = (uint32_t)(hi + WW + 1);
#pragma unroll
    for (int lev = 0; lev < 7; ++lev) {
        const uint32_t lk = (l + ((1u << lev) - 1u)) >> lev, hk = h >> lev;
        const bool go = lk < hk;
        r = unite(r, ut[go && (lk & 1u) ? lk : 0u]);
        r = unite(r, ut[go && (hk & 1u) ? hk - 1u : 0u]);
    }
    return r;
}

}  // namespace tb
