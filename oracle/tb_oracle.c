/*
 * libtreebbox ORACLE -- test infrastructure only.
 *
 * A plain, single-threaded, obviously-sequential CPU implementation of what
 * the GPU path computes.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header or table with the GPU path.
 *
 * What it follows (Levien, "Fast GPU bounding boxes on tree-structured
 * scenes", arXiv 2205.11659):
 *  - The sequential stack algorithm of Fig. 1 (section "The parentheses
 *    matching problem"): a stack seeded with -1; each element records the top
 *    of the stack, opens push their own index, closes pop.  `pm` below is
 *    exactly that output; `match` is the classical partner, which the same
 *    section says is reconstructed from it.
 *  - The Introduction's sequential bounding-box walk: each stack entry holds
 *    one clip box and one blend box; clip nodes intersect, blends union.
 *  - Node boxes per the Introduction: a leaf's box is its own box
 *    intersected with every clip node on its path to the root; a blend
 *    node's box is the union of all its descendant leaves (section
 *    "Parallel bounding boxes": clips first, then unions of clipped boxes;
 *    descendants are the slice between the open and the close).
 *  - The union is stored at the close and copied to the open (section "GPU
 *    implementation of clipping and blending", last paragraph).
 *
 * Readings where the paper is silent:
 *  - EMPTY = (+inf,+inf,-inf,-inf); a box is kept only if x0<x1 && y0<y1,
 *    otherwise it becomes EMPTY ("canon").  The whole-plane root clip context
 *    is INF = (-inf,-inf,+inf,+inf).
 *  - BEGIN_CLIP's box is canon(own box ∩ enclosing clip context); END_CLIP
 *    carries the box of its BEGIN_CLIP.  Blends pass the clip context through
 *    unchanged; only leaves enter unions.
 *  - Malformed input sets status bits; outputs are then unspecified.
 *  - Inputs are NaN-free and hold no -0.0.
 *
 * The reference gradient (tbo_backward) is not in the paper; its rule is
 * stated at that function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { LEAF = 0, BEGIN_CLIP = 1, END_CLIP = 2, BEGIN_BLEND = 3, END_BLEND = 4 };
enum { ST_BAD_KIND = 1u, ST_UNBALANCED = 2u, ST_KIND_MISMATCH = 4u };

typedef struct { float x0, y0, x1, y1; } box4;
typedef struct { double x0, y0, x1, y1; } box4d;

static float fmx(float a, float b) { return (b > a) ? b : a; }
static float fmn(float a, float b) { return (b < a) ? b : a; }
static double dmx(double a, double b) { return (b > a) ? b : a; }
static double dmn(double a, double b) { return (b < a) ? b : a; }

static box4 b_inf(void) { box4 r = {-INFINITY, -INFINITY, INFINITY, INFINITY}; return r; }
static box4 b_empty(void) { box4 r = {INFINITY, INFINITY, -INFINITY, -INFINITY}; return r; }
static box4 b_isect(box4 a, box4 b) {
    box4 r = {fmx(a.x0, b.x0), fmx(a.y0, b.y0), fmn(a.x1, b.x1), fmn(a.y1, b.y1)};
    return r;
}
static box4 b_union(box4 a, box4 b) {
    box4 r = {fmn(a.x0, b.x0), fmn(a.y0, b.y0), fmx(a.x1, b.x1), fmx(a.y1, b.y1)};
    return r;
}
static box4 b_canon(box4 a) { return (a.x0 < a.x1 && a.y0 < a.y1) ? a : b_empty(); }

static box4d d_inf(void) { box4d r = {-INFINITY, -INFINITY, INFINITY, INFINITY}; return r; }
static box4d d_empty(void) { box4d r = {INFINITY, INFINITY, -INFINITY, -INFINITY}; return r; }
static box4d d_isect(box4d a, box4d b) {
    box4d r = {dmx(a.x0, b.x0), dmx(a.y0, b.y0), dmn(a.x1, b.x1), dmn(a.y1, b.y1)};
    return r;
}
static box4d d_union(box4d a, box4d b) {
    box4d r = {dmn(a.x0, b.x0), dmn(a.y0, b.y0), dmx(a.x1, b.x1), dmx(a.y1, b.y1)};
    return r;
}
static box4d d_canon(box4d a) { return (a.x0 < a.x1 && a.y0 < a.y1) ? a : d_empty(); }

/* One stack entry of the sequential walk: the open's index and kind, the
   clip box its children see, and the blend (union) box accumulated so far. */
typedef struct {
    int64_t idx;
    uint32_t kind;
    box4 clip, acc;
} entry;

typedef struct {
    int64_t idx;
    uint32_t kind;
    box4d clip, acc;
} entryd;

/*
 * Forward: match, pm (nullable), out (nullable; 4 floats per row).
 * kind: n values; box: 4n floats (x0,y0,x1,y1 per row).
 * Returns the status bits.
 */
uint32_t tbo_bbox(const uint32_t *kind, const float *box, int64_t n, int32_t *match, int32_t *pm,
                  float *out) {
    uint32_t status = 0;
    entry *S = (entry *)malloc(sizeof(entry) * (size_t)(n + 1));
    if (!S) return 0xFFFFFFFFu;
    int64_t sp = 0;
    S[sp].idx = -1;
    S[sp].kind = 0xFFFFFFFFu; /* root */
    S[sp].clip = b_inf();
    S[sp].acc = b_empty();
    sp = 1;
    box4 *o = (box4 *)out;
    const box4 *bx = (const box4 *)box;
    for (int64_t i = 0; i < n; ++i) {
        entry *t = &S[sp - 1];
        if (pm) pm[i] = (int32_t)t->idx;
        if (match) match[i] = -1;
        uint32_t k = kind[i];
        if (k > 4) {
            status |= ST_BAD_KIND;
            if (o) o[i] = b_empty();
            continue;
        }
        if (k == LEAF) {
            box4 b = box ? b_canon(b_isect(bx[i], t->clip)) : b_empty();
            if (o) o[i] = b;
            t->acc = b_union(t->acc, b);
        } else if (k == BEGIN_CLIP) {
            box4 c = box ? b_canon(b_isect(bx[i], t->clip)) : b_empty();
            if (o) o[i] = c;
            S[sp].idx = i;
            S[sp].kind = BEGIN_CLIP;
            S[sp].clip = c;
            S[sp].acc = b_empty();
            ++sp;
        } else if (k == BEGIN_BLEND) {
            S[sp].idx = i;
            S[sp].kind = BEGIN_BLEND;
            S[sp].clip = t->clip;
            S[sp].acc = b_empty();
            ++sp;
        } else { /* END_CLIP or END_BLEND */
            if (t->idx == -1) {
                status |= ST_UNBALANCED; /* would pop the root */
                if (o) o[i] = b_empty();
                continue;
            }
            if ((k == END_CLIP) != (t->kind == BEGIN_CLIP)) status |= ST_KIND_MISMATCH;
            entry e = S[--sp];
            if (match) {
                match[i] = (int32_t)e.idx;
                match[e.idx] = (int32_t)i;
            }
            if (o) {
                if (e.kind == BEGIN_BLEND) {
                    o[e.idx] = e.acc;
                    o[i] = e.acc;
                } else {
                    o[i] = o[e.idx];
                }
            }
            S[sp - 1].acc = b_union(S[sp - 1].acc, e.acc);
        }
    }
    if (sp != 1) status |= ST_UNBALANCED;
    free(S);
    return status;
}

/* Matching only (kinds): same walk without boxes. */
uint32_t tbo_match(const uint32_t *kind, int64_t n, int32_t *match, int32_t *pm) {
    return tbo_bbox(kind, NULL, n, match, pm, NULL);
}

/*
 * fp32 affine transforms composed down the tree, a monoid whose products
 * round, so the combine order is part of the definition.  The order is that
 * of pointer jumping (section "Parallel bounding boxes", Clips): every open
 * holds a value and a pointer to its enclosing open; in each round all of
 * them at once replace value v by (value at the pointer) . v and the pointer
 * by the pointer's pointer, reading the previous round's arrays, until no
 * pointer is left.  After round r an open holds the product over itself and
 * its 2^r - 1 nearest enclosing opens, outermost first.  Leaves take the
 * final value of the open enclosing them (the identity at the root) and a
 * close that of its open.
 *
 * Product p.q (q applied first), every operation an fp32 operation rounded
 * to nearest even, no fused multiply-add:
 *   a = p.a*q.a + p.b*q.d          b = p.a*q.b + p.b*q.e
 *   c = (p.a*q.c + p.b*q.f) + p.c
 *   d = p.d*q.a + p.e*q.d          e = p.d*q.b + p.e*q.e
 *   f = (p.d*q.c + p.e*q.f) + p.f
 * (each x*y rounded, then each + rounded, left to right as written).
 * Status: as tbo_match (kind pairs are not checked).
 */
typedef struct { float a, b, c, d, e, f; } aff32;
static aff32 aff32_id(void) { aff32 r = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f}; return r; }
static float mul_rn(float x, float y) { volatile float r = x * y; return r; }
static float add_rn(float x, float y) { volatile float r = x + y; return r; }
static aff32 aff32_mul(aff32 p, aff32 q) {
    aff32 r;
    r.a = add_rn(mul_rn(p.a, q.a), mul_rn(p.b, q.d));
    r.b = add_rn(mul_rn(p.a, q.b), mul_rn(p.b, q.e));
    r.c = add_rn(add_rn(mul_rn(p.a, q.c), mul_rn(p.b, q.f)), p.c);
    r.d = add_rn(mul_rn(p.d, q.a), mul_rn(p.e, q.d));
    r.e = add_rn(mul_rn(p.d, q.b), mul_rn(p.e, q.e));
    r.f = add_rn(add_rn(mul_rn(p.d, q.c), mul_rn(p.e, q.f)), p.f);
    return r;
}

uint32_t tbo_compose_f32(const uint32_t *kind, const float *xf, int64_t n, float *out) {
    const size_t m = (size_t)(n > 0 ? n : 1);
    int32_t *pm = (int32_t *)malloc(sizeof(int32_t) * m);
    aff32 *val = (aff32 *)malloc(sizeof(aff32) * m), *nval = (aff32 *)malloc(sizeof(aff32) * m);
    int64_t *ptr = (int64_t *)malloc(sizeof(int64_t) * m), *nptr = (int64_t *)malloc(sizeof(int64_t) * m);
    if (!pm || !val || !nval || !ptr || !nptr) return 0x80000000u;
    const uint32_t status = tbo_match(kind, n, NULL, pm);
    int any = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int open = kind[i] == BEGIN_CLIP || kind[i] == BEGIN_BLEND;
        const float *x = xf + 6 * i;
        aff32 own = {x[0], x[1], x[2], x[3], x[4], x[5]};
        val[i] = open ? own : aff32_id();
        ptr[i] = open ? pm[i] : -1;
        any |= ptr[i] >= 0;
    }
    while (any) { /* one round: every pointer at once, from the previous arrays */
        any = 0;
        for (int64_t i = 0; i < n; ++i) {
            const int64_t p = ptr[i];
            if (p >= 0) {
                nval[i] = aff32_mul(val[p], val[i]);
                nptr[i] = ptr[p];
            } else {
                nval[i] = val[i];
                nptr[i] = -1;
            }
            any |= nptr[i] >= 0;
        }
        aff32 *tv = val; val = nval; nval = tv;
        int64_t *tp = ptr; ptr = nptr; nptr = tp;
    }
    for (int64_t i = 0; i < n; ++i) {
        const int open = kind[i] == BEGIN_CLIP || kind[i] == BEGIN_BLEND;
        const aff32 o = open ? val[i] : pm[i] >= 0 ? val[pm[i]] : aff32_id();
        float *y = out + 6 * i;
        y[0] = o.a, y[1] = o.b, y[2] = o.c, y[3] = o.d, y[4] = o.e, y[5] = o.f;
    }
    free(pm), free(val), free(nval), free(ptr), free(nptr);
    return status;
}

/*
 * fp32 transforms combined UP the tree: an open (and its close) gets the
 * ordered product of the transforms of the leaves strictly between them,
 * in sequence order, the leftmost leaf the leftmost factor (p.q as in
 * tbo_compose_f32); an open with no leaf inside gets the identity; a leaf
 * gets its own transform.  Products round, so the grouping is fixed: that
 * of a segment tree over the positions.  With N the smallest power of two
 * >= n, node N+i holds element i's transform if it is a leaf and nothing
 * otherwise, node v combines nodes 2v and 2v+1 (a missing side leaves the
 * other unchanged), and a range [lo, hi] is answered bottom-up:
 *   l = lo+N, r = hi+N+1, L = R = nothing;
 *   while l < r: if l odd, L = L.node[l++]; if r odd, R = node[--r].R;
 *                l /= 2, r /= 2;
 *   result L.R.
 * Status: as tbo_match.
 */
typedef struct { aff32 v; int some; } aff32o; /* some = 0: no leaf */
static aff32o comb32(aff32o a, aff32o b) {
    if (!a.some) return b;
    if (!b.some) return a;
    aff32o r = {aff32_mul(a.v, b.v), 1};
    return r;
}

uint32_t tbo_reduce_up_f32(const uint32_t *kind, const float *xf, int64_t n, float *out) {
    const size_t m = (size_t)(n > 0 ? n : 1);
    int32_t *match = (int32_t *)malloc(sizeof(int32_t) * m);
    int64_t N = 1;
    while (N < n) N <<= 1;
    aff32o *node = (aff32o *)calloc((size_t)(2 * N), sizeof(aff32o));
    if (!match || !node) return 0x80000000u;
    const uint32_t status = tbo_match(kind, n, match, NULL);
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != LEAF) continue;
        const float *x = xf + 6 * i;
        aff32o leaf = {{x[0], x[1], x[2], x[3], x[4], x[5]}, 1};
        node[N + i] = leaf;
    }
    for (int64_t v = N - 1; v >= 1; --v) node[v] = comb32(node[2 * v], node[2 * v + 1]);
    for (int64_t i = 0; i < n; ++i) {
        aff32 o = aff32_id();
        if (kind[i] == LEAF) {
            o = node[N + i].v;
        } else if ((kind[i] == BEGIN_CLIP || kind[i] == BEGIN_BLEND) && match[i] > i) {
            aff32o L = {aff32_id(), 0}, R = {aff32_id(), 0};
            int64_t l = i + 1 + N, r = (int64_t)match[i] - 1 + N + 1;
            while (l < r) {
                if (l & 1) L = comb32(L, node[l++]);
                if (r & 1) R = comb32(node[--r], R);
                l >>= 1;
                r >>= 1;
            }
            const aff32o q = comb32(L, R);
            if (q.some) o = q.v;
        } else if ((kind[i] == END_CLIP || kind[i] == END_BLEND) && match[i] >= 0 && match[i] < i) {
            continue; /* written with its open below */
        }
        float *y = out + 6 * i;
        y[0] = o.a, y[1] = o.b, y[2] = o.c, y[3] = o.d, y[4] = o.e, y[5] = o.f;
        if ((kind[i] == BEGIN_CLIP || kind[i] == BEGIN_BLEND) && match[i] > i)
            memcpy(out + 6 * (int64_t)match[i], y, 6 * sizeof(float));
    }
    free(match), free(node);
    return status;
}

/*
 * Matching over typed brackets (section "The parentheses matching problem",
 * Fig. 1, with several kinds of parentheses as parsing needs them).
 * Token 0 is not a bracket; an odd token 2t+1 opens a bracket of type t, an
 * even token 2t+2 closes one.  Tokens 0..4 are exactly the five element
 * kinds (types 0 and 1 being clip and blend), so on them this equals
 * tbo_match.  The walk is Fig. 1's stack; a close whose type differs from
 * its open's sets KIND_MISMATCH and still matches that open; a close with
 * nothing open, or an open never closed, sets UNBALANCED.  Every uint32 is
 * a valid token (no BAD_KIND).
 */
uint32_t tbo_match_brackets(const uint32_t *tok, int64_t n, int32_t *match, int32_t *pm) {
    uint32_t status = 0;
    int64_t *S = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!S) return 0xFFFFFFFFu;
    int64_t sp = 0;
    S[sp++] = -1; /* the root */
    for (int64_t i = 0; i < n; ++i) {
        const int64_t top = S[sp - 1];
        if (pm) pm[i] = (int32_t)top;
        if (match) match[i] = -1;
        const uint32_t k = tok[i];
        if (k == 0) continue;
        if (k & 1u) {
            S[sp++] = i;
            continue;
        }
        if (top == -1) {
            status |= ST_UNBALANCED;
            continue;
        }
        if (tok[top] + 1u != k) status |= ST_KIND_MISMATCH;
        --sp;
        if (match) {
            match[i] = (int32_t)top;
            match[top] = (int32_t)i;
        }
    }
    if (sp != 1) status |= ST_UNBALANCED;
    free(S);
    return status;
}

/* The same forward walk in fp64 (for finite-difference checks). */
uint32_t tbo_bbox_f64(const uint32_t *kind, const double *box, int64_t n, double *out) {
    uint32_t status = 0;
    entryd *S = (entryd *)malloc(sizeof(entryd) * (size_t)(n + 1));
    if (!S) return 0xFFFFFFFFu;
    int64_t sp = 0;
    S[0].idx = -1;
    S[0].kind = 0xFFFFFFFFu;
    S[0].clip = d_inf();
    S[0].acc = d_empty();
    sp = 1;
    box4d *o = (box4d *)out;
    const box4d *bx = (const box4d *)box;
    for (int64_t i = 0; i < n; ++i) {
        entryd *t = &S[sp - 1];
        uint32_t k = kind[i];
        if (k > 4) {
            status |= ST_BAD_KIND;
            o[i] = d_empty();
            continue;
        }
        if (k == LEAF) {
            box4d b = d_canon(d_isect(bx[i], t->clip));
            o[i] = b;
            t->acc = d_union(t->acc, b);
        } else if (k == BEGIN_CLIP) {
            box4d c = d_canon(d_isect(bx[i], t->clip));
            o[i] = c;
            S[sp].idx = i;
            S[sp].kind = BEGIN_CLIP;
            S[sp].clip = c;
            S[sp].acc = d_empty();
            ++sp;
        } else if (k == BEGIN_BLEND) {
            S[sp].idx = i;
            S[sp].kind = BEGIN_BLEND;
            S[sp].clip = t->clip;
            S[sp].acc = d_empty();
            ++sp;
        } else {
            if (t->idx == -1) {
                status |= ST_UNBALANCED;
                o[i] = d_empty();
                continue;
            }
            if ((k == END_CLIP) != (t->kind == BEGIN_CLIP)) status |= ST_KIND_MISMATCH;
            entryd e = S[--sp];
            if (e.kind == BEGIN_BLEND) {
                o[e.idx] = e.acc;
                o[i] = e.acc;
            } else {
                o[i] = o[e.idx];
            }
            S[sp - 1].acc = d_union(S[sp - 1].acc, e.acc);
        }
    }
    if (sp != 1) status |= ST_UNBALANCED;
    free(S);
    return status;
}

/*
 * Reference gradient (not in the paper).
 *
 * Every output coordinate is a max or min of input coordinates, so its
 * gradient goes to one input coordinate, its "source":
 *  - LEAF or BEGIN_CLIP row o, coordinate c: the candidates are o itself and
 *    every BEGIN_CLIP enclosing o; those whose box[.][c] equals out[o][c]
 *    attain it, and the source is the lowest element index among them.
 *  - END_CLIP: the source of its BEGIN_CLIP.
 *  - BEGIN_BLEND / END_BLEND: among the descendant leaves l with out[l] not
 *    EMPTY and out[l][c] == out[o][c], the sources src(l, c); the lowest
 *    element index among those.
 *  - Rows whose out is EMPTY route nothing.
 * grad_in[src][c] accumulates q(g) = round-half-even(g * 2^32) as an exact
 * 64-bit integer (order cannot change an integer sum), and is then rounded
 * once to fp32: grad_in = RNE_fp32(sum) * 2^-32.  q(g) rounds every g to a
 * multiple of 2^-32, so a contribution with |g| < 2^-9 (fewer than 24
 * significant bits left on that grid) is not exact, and |g| <= 2^-33 counts
 * as 0.  Sums wrap modulo 2^64; precondition: the final sum fits in an
 * int64 (|sum of g| < 2^31).  Rows never attained get 0.
 *
 * Written as the definition: every leaf/clip row walks its whole ancestor
 * chain, every blend row visits every row of its slice.
 */
static void sources(const uint32_t *kind, const float *box, int64_t n, const int32_t *match,
                    const int32_t *pm, const float *out, int64_t *src) {
    for (int64_t o = 0; o < n; ++o) {
        for (int c = 0; c < 4; ++c) src[4 * o + c] = -1;
        uint32_t k = kind[o];
        if (k != LEAF && k != BEGIN_CLIP) continue;
        const float *ov = out + 4 * o;
        if (!(ov[0] < ov[2] && ov[1] < ov[3])) continue; /* EMPTY */
        for (int c = 0; c < 4; ++c) {
            int64_t best = (box[4 * o + c] == ov[c]) ? o : -1;
            /* ancestors come in decreasing index order: the last hit is the lowest */
            for (int64_t a = pm[o]; a >= 0; a = pm[a])
                if (kind[a] == BEGIN_CLIP && box[4 * a + c] == ov[c]) best = a;
            src[4 * o + c] = best;
        }
    }
    for (int64_t o = 0; o < n; ++o)
        if (kind[o] == END_CLIP && match[o] >= 0)
            for (int c = 0; c < 4; ++c) src[4 * o + c] = src[4 * match[o] + c];
    for (int64_t o = 0; o < n; ++o) {
        if (kind[o] != END_BLEND || match[o] < 0) continue;
        int64_t op = match[o];
        const float *ov = out + 4 * o;
        int64_t best[4] = {-1, -1, -1, -1};
        if (ov[0] < ov[2] && ov[1] < ov[3]) {
            for (int64_t l = op + 1; l < o; ++l) {
                if (kind[l] != LEAF) continue;
                const float *lv = out + 4 * l;
                if (!(lv[0] < lv[2] && lv[1] < lv[3])) continue;
                for (int c = 0; c < 4; ++c) {
                    if (lv[c] != ov[c]) continue;
                    int64_t s = src[4 * l + c];
                    if (best[c] < 0 || s < best[c]) best[c] = s;
                }
            }
        }
        for (int c = 0; c < 4; ++c) src[4 * o + c] = src[4 * op + c] = best[c];
    }
}

/* Sources per output coordinate (4n int64, -1 where nothing routes). */
uint32_t tbo_sources(const uint32_t *kind, const float *box, int64_t n, int64_t *src) {
    size_t m = (size_t)(n > 0 ? n : 1);
    int32_t *match = (int32_t *)malloc(sizeof(int32_t) * m);
    int32_t *pm = (int32_t *)malloc(sizeof(int32_t) * m);
    float *out = (float *)malloc(sizeof(float) * 4 * m);
    if (!match || !pm || !out) return 0xFFFFFFFFu;
    uint32_t status = tbo_bbox(kind, box, n, match, pm, out);
    if (!status) sources(kind, box, n, match, pm, out, src);
    free(match), free(pm), free(out);
    return status;
}

/* q(g) is defined for |g| < 2^31 only (g * 2^32 must fit in an int64); a
   routed coordinate whose upstream gradient lies outside that range, or is
   NaN, sets this status bit instead of contributing. */
enum { ST_GRAD_RANGE = 16u };

uint32_t tbo_backward(const uint32_t *kind, const float *box, const float *grad_out, int64_t n,
                      float *grad_in) {
    size_t m = (size_t)(n > 0 ? n : 1);
    int64_t *src = (int64_t *)malloc(sizeof(int64_t) * 4 * m);
    /* sums wrap modulo 2^64 (unsigned), so only the final sum must fit */
    uint64_t *acc = (uint64_t *)calloc(4 * m, sizeof(uint64_t));
    if (!src || !acc) return 0xFFFFFFFFu;
    uint32_t status = tbo_sources(kind, box, n, src);
    if (!status) {
        for (int64_t o = 0; o < n; ++o)
            for (int c = 0; c < 4; ++c) {
                int64_t s = src[4 * o + c];
                if (s < 0) continue;
                float gf = grad_out[4 * o + c];
                if (!(fabsf(gf) < 2147483648.0f)) {
                    status |= ST_GRAD_RANGE;
                    continue;
                }
                double g = (double)gf * 4294967296.0; /* exact scaling */
                acc[4 * s + c] += (uint64_t)llrint(g);
            }
    }
    for (int64_t i = 0; i < 4 * n; ++i) grad_in[i] = (float)(int64_t)acc[i] * 0x1p-32f;
    free(src), free(acc);
    return status;
}

/*
 * Composition of a transform monoid down the tree (the Introduction names
 * transforms composed down a skeleton as an application of the same method
 * to a general monoid).  Every open carries a 2-D affine transform
 * [a b c; d e f] on integer coordinates, arithmetic modulo 2^32 (exact, so
 * associative, and not commutative).  Element i's output is the product of
 * the transforms of all opens enclosing it, outermost first; an open's
 * output includes its own transform, and a close's output is its open's.
 * Leaves' and closes' input rows are ignored.  Both open kinds carry a
 * transform and closes pop either kind (kind pairs are not checked).
 * Walk: the stack of Fig. 1, each entry holding the product down to it.
 */
typedef struct { uint32_t a, b, c, d, e, f; } aff;

static aff aff_id(void) { aff r = {1u, 0u, 0u, 0u, 1u, 0u}; return r; }
/* p . q : apply q first, then p */
static aff aff_mul(aff p, aff q) {
    aff r;
    r.a = p.a * q.a + p.b * q.d;
    r.b = p.a * q.b + p.b * q.e;
    r.c = p.a * q.c + p.b * q.f + p.c;
    r.d = p.d * q.a + p.e * q.d;
    r.e = p.d * q.b + p.e * q.e;
    r.f = p.d * q.c + p.e * q.f + p.f;
    return r;
}

uint32_t tbo_compose(const uint32_t *kind, const uint32_t *xf, int64_t n, uint32_t *out) {
    uint32_t status = 0;
    aff *S = (aff *)malloc(sizeof(aff) * (size_t)(n + 1));
    if (!S) return 0x80000000u;
    int64_t sp = 0;
    S[sp++] = aff_id(); /* the root: nothing applied */
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t k = kind[i];
        aff o = S[sp - 1];
        if (k > END_BLEND) {
            status |= ST_BAD_KIND;
        } else if (k == BEGIN_CLIP || k == BEGIN_BLEND) {
            const uint32_t *x = xf + 6 * i;
            aff own = {x[0], x[1], x[2], x[3], x[4], x[5]};
            o = aff_mul(S[sp - 1], own);
            S[sp++] = o;
        } else if (k == END_CLIP || k == END_BLEND) {
            if (sp == 1) {
                status |= ST_UNBALANCED;
            } else {
                o = S[--sp];
            }
        }
        uint32_t *y = out + 6 * i;
        y[0] = o.a, y[1] = o.b, y[2] = o.c, y[3] = o.d, y[4] = o.e, y[5] = o.f;
    }
    if (sp != 1) status |= ST_UNBALANCED;
    free(S);
    return status;
}

/*
 * Draw-object stream front end (Introduction: the renderer first extracts
 * just the clip and blend elements of its scene description by stream
 * compaction, a prefix-sum application, and runs the bounding-box
 * algorithm on the extracted sequence only).  Here the stream holds the
 * tree's elements (tags 0..4: leaves take part in blend unions, so they are
 * extracted too) among elements outside the tree (tag 5).
 *   1. compaction: the tree elements, in stream order, with their positions;
 *   2. the sequential walk (tbo_bbox) on the compacted sequence;
 *   3. each result goes back to its element's stream position, and each
 *      partner index is translated to a stream position.
 * Rows and match entries at tag-5 positions are left as they were.  A tag
 * above 5 raises BAD_KIND and is dropped like tag 5.
 */
enum { STREAM_OTHER = 5 };

uint32_t tbo_bbox_stream(const uint32_t *tag, const float *box, int64_t n, int32_t *match,
                         float *out) {
    uint32_t status = 0;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (tag[i] <= END_BLEND) ++m;
        else if (tag[i] != STREAM_OTHER) status |= ST_BAD_KIND;
    }
    const size_t mm = (size_t)(m > 0 ? m : 1);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * mm);
    uint32_t *ck = (uint32_t *)malloc(sizeof(uint32_t) * mm);
    float *cb = (float *)malloc(sizeof(float) * 4 * mm);
    int32_t *cm = (int32_t *)malloc(sizeof(int32_t) * mm);
    float *co = (float *)malloc(sizeof(float) * 4 * mm);
    if (!pos || !ck || !cb || !cm || !co) {
        free(pos), free(ck), free(cb), free(cm), free(co);
        return 0x80000000u;
    }
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) { /* 1 */
        if (tag[i] > END_BLEND) continue;
        pos[j] = i;
        ck[j] = tag[i];
        memcpy(cb + 4 * j, box + 4 * i, 4 * sizeof(float));
        ++j;
    }
    status |= tbo_bbox(ck, cb, m, cm, NULL, co); /* 2 */
    for (j = 0; j < m; ++j) {                    /* 3 */
        const int64_t i = pos[j];
        if (match) match[i] = cm[j] >= 0 ? (int32_t)pos[cm[j]] : -1;
        if (out) memcpy(out + 4 * i, co + 4 * j, 4 * sizeof(float));
    }
    free(pos), free(ck), free(cb), free(cm), free(co);
    return status;
}
