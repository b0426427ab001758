/*
 * Seeded synthetic scene generator.
 *
 * Produces flattened scene trees: a node with children is written as an
 * open element, its children, then a close element (the flattened encoding
 * of the paper's Introduction / Motivation).  Element kinds:
 *   0 LEAF, 1 BEGIN_CLIP, 2 END_CLIP, 3 BEGIN_BLEND, 4 END_BLEND.
 * Rows for LEAF and BEGIN_CLIP carry an fp32 box (x0, y0, x1, y1); every
 * other row is zero.
 *
 * The sequence shape follows the paper's workload (Performance results):
 * pushes and pops equally likely unless a pop would underflow, here with a
 * depth cap and leaves in between.  This module only draws inputs; it holds
 * none of the bounding-box arithmetic (no intersection or union is formed
 * here), and both the oracle and the GPU path consume what it writes.
 *
 * Random numbers: xoshiro256** seeded through splitmix64, both from their
 * published definitions (Blackman & Vigna, "Scrambled linear pseudorandom
 * number generators", 2018/2021; splitmix64 from Steele, Lea & Flood 2014).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_LEAF = 0, K_BCLIP = 1, K_ECLIP = 2, K_BBLEND = 3, K_EBLEND = 4 };

/* ------------------------------------------------------------------ rng */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t tbg_splitmix64(uint64_t x) {
    uint64_t s = x;
    return splitmix64_next(&s);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64_next(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}

/* uniform double in [0, 1) with 53 random bits */
static inline double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* exponential with the given mean */
static inline double rng_exp(rng_t *r, double mean) { return -mean * log(1.0 - rng_u01(r)); }

/* integer uniform in [lo, hi] */
static inline int64_t rng_int(rng_t *r, int64_t lo, int64_t hi) {
    return lo + (int64_t)(rng_u01(r) * (double)(hi - lo + 1));
}

/* ------------------------------------------------------------ builder */
enum { BOX_INDEP = 0, BOX_NESTED = 1, BOX_GRID = 2, BOX_NESTED_ALL = 3, BOX_INSET = 4,
       BOX_INSET_ND = 5 };

typedef struct {
    uint32_t *kind;
    float *box;
    int64_t n, pos;
    int64_t *stk;      /* positions of currently open elements */
    int64_t *clipanc;  /* per stack level: position of nearest clip at or below it, or -1 */
    int64_t *reg;      /* BOX_INSET*: per stack level, 4 grid coordinates of the region
                          its children are drawn in */
    int64_t sp, cap_stk;
    int box_mode;
    double p_disjoint; /* BOX_NESTED, BOX_INSET: probability that a clip misses its parent */
    int in_chain;      /* BOX_INSET*: the opens being emitted form a nested chain */
    int chain_first;   /* ... and the chain's first clip is still to come */
    rng_t r;
} builder;

static int b_init(builder *b, uint32_t *kind, float *box, int64_t n, int64_t max_depth,
                  uint64_t seed, int box_mode) {
    b->kind = kind;
    b->box = box;
    b->n = n;
    b->pos = 0;
    b->cap_stk = max_depth + 2;
    b->stk = (int64_t *)malloc(sizeof(int64_t) * (size_t)b->cap_stk);
    b->clipanc = (int64_t *)malloc(sizeof(int64_t) * (size_t)b->cap_stk);
    b->reg = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)b->cap_stk);
    if (!b->stk || !b->clipanc || !b->reg) return -1;
    b->sp = 0;
    b->box_mode = box_mode;
    b->p_disjoint = box_mode == BOX_INSET_ND ? 0.0 : 0.05;
    b->in_chain = 0;
    b->chain_first = 0;
    rng_seed(&b->r, seed);
    return 0;
}

static void b_free(builder *b) {
    free(b->stk);
    free(b->clipanc);
    free(b->reg);
}

/*
 * BOX_INSET / BOX_INSET_ND: value-rich nested boxes on a 2^-8 grid (all
 * coordinates are integers times 2^-8 below 2^13 in magnitude, so exact in
 * fp32).  Every node's box is drawn around an inner box that lies inside
 * the region of its nearest clip ancestor; a clip's inner box is the region
 * of its own subtree.  Regions therefore nest, so every clip context and
 * every leaf stays non-empty, while each drawn box sticks out of the region
 * on some sides and is cut there by some ancestor clip.  The generator only
 * draws sub-intervals of intervals; it forms no intersection or union.
 *  - Root region: [256, 3840]^2.
 *  - Leaf: inner box of size Exp(64) (at least one grid step, at most the
 *    region) at a uniform position in the region; it sticks out on x0 with
 *    probability 1/8, on x1 and y1 with probability 1/2 (by 1 + Exp(16)
 *    capped at 255 units), never on y0.
 *  - Clip in a walk: inner box of U[1/2, 1) times the region's size at a
 *    uniform position; sticks out on each side with probability 1/2.  With
 *    probability p_disjoint (BOX_INSET: 0.05, BOX_INSET_ND: 0) the clip is
 *    moved 8192 units left, away from every other box, so its subtree is
 *    empty.
 *  - Clip in a nested chain: the inner box is the region with side c moved
 *    in by one grid step with probability 1/256, 1/4096, 1/65536, 0 for
 *    x0, y0, x1, y1 (a side moved in is "tight": the clip does not stick out
 *    there); the chain's first clip is tight on all sides; other sides stick
 *    out by 1 + Exp(4) units.  So the running clip context along a chain is
 *    set by the latest tight clip on each side, which on y1 is the chain's
 *    first clip, however deep the chain.
 */
#define INSET_G 256.0 /* grid steps per unit */

static int64_t g_ext(rng_t *r, double mean_units) {
    double e = floor(rng_exp(r, mean_units) * INSET_G);
    if (e > 254.0 * INSET_G) e = 254.0 * INSET_G;
    return (int64_t)INSET_G + (int64_t)e;
}

/* the region children of the current top are drawn in (a blend level holds
   its parent's region) */
static void inset_region(builder *b, int64_t rg[4]) {
    if (b->sp > 0) {
        memcpy(rg, b->reg + 4 * (b->sp - 1), 4 * sizeof(int64_t));
    } else {
        rg[0] = rg[1] = (int64_t)(256 * INSET_G);
        rg[2] = rg[3] = (int64_t)(3840 * INSET_G);
    }
}

/* a sub-interval of [lo, hi] of length len (1 <= len <= hi - lo), uniform */
static int64_t g_place(rng_t *r, int64_t lo, int64_t hi, int64_t len) {
    return lo + (int64_t)floor(rng_u01(r) * (double)(hi - lo - len + 1));
}

static void inset_store(float *dst, const int64_t c[4]) {
    for (int q = 0; q < 4; ++q) dst[q] = (float)((double)c[q] / INSET_G);
}

/* draws element i (a leaf or a clip open); a clip's inner box goes to inner */
static void draw_inset(builder *b, uint32_t k, float *dst, int64_t inner[4]) {
    rng_t *r = &b->r;
    int64_t rg[4], in[4], c[4];
    inset_region(b, rg);
    const int64_t rw = rg[2] - rg[0], rh = rg[3] - rg[1];
    if (k == K_LEAF) {
        int64_t w = (int64_t)ceil(rng_exp(r, 64.0) * INSET_G), h = (int64_t)ceil(rng_exp(r, 64.0) * INSET_G);
        if (w < 1) w = 1;
        if (h < 1) h = 1;
        if (w > rw) w = rw;
        if (h > rh) h = rh;
        in[0] = g_place(r, rg[0], rg[2], w);
        in[1] = g_place(r, rg[1], rg[3], h);
        in[2] = in[0] + w;
        in[3] = in[1] + h;
        c[0] = in[0] - (rng_u01(r) < 0.125 ? g_ext(r, 16.0) : 0);
        c[1] = in[1];
        c[2] = in[2] + (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        c[3] = in[3] + (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        inset_store(dst, c);
        return;
    }
    if (b->in_chain) {
        static const double p_tight[4] = {1.0 / 256, 1.0 / 4096, 1.0 / 65536, 0.0};
        const int first = b->chain_first;
        b->chain_first = 0;
        for (int q = 0; q < 4; ++q) {
            const int lowside = q < 2;
            const int64_t span = rg[q < 2 ? q + 2 : q] - rg[q < 2 ? q : q - 2];
            int tight = first;
            in[q] = rg[q];
            if (rng_u01(r) < p_tight[q] && span > 4) {
                in[q] += lowside ? 1 : -1;
                tight = 1;
            }
            const int64_t e = tight ? 0 : g_ext(r, 4.0);
            c[q] = lowside ? in[q] - e : in[q] + e;
        }
        /* a side moves in only while the region spans more than 4 steps, so
           the inner box keeps at least 3 steps per axis */
    } else {
        int64_t w = (int64_t)floor((double)rw * (0.5 + 0.5 * rng_u01(r)));
        int64_t h = (int64_t)floor((double)rh * (0.5 + 0.5 * rng_u01(r)));
        if (w < 1) w = 1;
        if (h < 1) h = 1;
        in[0] = g_place(r, rg[0], rg[2], w);
        in[1] = g_place(r, rg[1], rg[3], h);
        in[2] = in[0] + w;
        in[3] = in[1] + h;
        c[0] = in[0] - (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        c[1] = in[1] - (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        c[2] = in[2] + (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        c[3] = in[3] + (rng_u01(r) < 0.5 ? g_ext(r, 16.0) : 0);
        /* (inside an already disjoint subtree every box is empty anyway) */
        if (rng_u01(r) < b->p_disjoint && rg[0] >= 0) {
            const int64_t shift = (int64_t)(8192 * INSET_G);
            c[0] -= shift, c[2] -= shift, in[0] -= shift, in[2] -= shift;
        }
    }
    memcpy(inner, in, sizeof in);
    inset_store(dst, c);
}

static void draw_box(builder *b, float *dst) {
    rng_t *r = &b->r;
    int64_t anc = b->sp > 0 ? b->clipanc[b->sp - 1] : -1;
    if (b->box_mode == BOX_GRID) {
        /* coordinates on a 2^-8 grid in [0, 4096); sizes exponential (mean 64)
           rounded up to the grid, at least one grid step; all exact in fp32 */
        double x0 = floor(rng_u01(r) * 1048576.0) / 256.0;
        double y0 = floor(rng_u01(r) * 1048576.0) / 256.0;
        double w = ceil(rng_exp(r, 64.0) * 256.0);
        double h = ceil(rng_exp(r, 64.0) * 256.0);
        if (w < 1.0) w = 1.0;
        if (h < 1.0) h = 1.0;
        dst[0] = (float)x0;
        dst[1] = (float)y0;
        dst[2] = (float)(x0 + w / 256.0);
        dst[3] = (float)(y0 + h / 256.0);
        return;
    }
    double w = rng_exp(r, 64.0), h = rng_exp(r, 64.0);
    float x0, y0;
    if ((b->box_mode == BOX_NESTED || b->box_mode == BOX_NESTED_ALL) && anc >= 0) {
        const float *a = b->box + 4 * anc;
        if (rng_u01(r) < b->p_disjoint) {
            /* shifted past the ancestor's right edge: disjoint from it */
            x0 = (float)((double)a[2] + 1.0 + rng_u01(r) * 64.0);
            y0 = (float)((double)a[1] + rng_u01(r) * ((double)a[3] - (double)a[1]));
        } else {
            /* overlapping the ancestor's box */
            x0 = (float)((double)a[0] - w + rng_u01(r) * ((double)a[2] - (double)a[0] + w));
            y0 = (float)((double)a[1] - h + rng_u01(r) * ((double)a[3] - (double)a[1] + h));
        }
    } else {
        x0 = (float)(rng_u01(r) * 4096.0);
        y0 = (float)(rng_u01(r) * 4096.0);
    }
    dst[0] = x0;
    dst[1] = y0;
    dst[2] = (float)((double)x0 + w);
    dst[3] = (float)((double)y0 + h);
}

static void b_emit(builder *b, uint32_t k) {
    int64_t i = b->pos++;
    b->kind[i] = k;
    float *dst = b->box + 4 * i;
    dst[0] = dst[1] = dst[2] = dst[3] = 0.0f;
    const int inset = b->box_mode == BOX_INSET || b->box_mode == BOX_INSET_ND;
    int64_t inner[4] = {0, 0, 0, 0};
    if (inset && (k == K_LEAF || k == K_BCLIP)) {
        draw_inset(b, k, dst, inner);
    } else if (k == K_LEAF || k == K_BCLIP) {
        if (b->box_mode == BOX_NESTED && k == K_LEAF) {
            /* BOX_NESTED: leaves keep the independent draw, only clips nest;
               BOX_NESTED_ALL nests leaves too */
            int save = b->box_mode;
            b->box_mode = BOX_INDEP;
            draw_box(b, dst);
            b->box_mode = save;
        } else {
            draw_box(b, dst);
        }
    }
    if (k == K_BCLIP || k == K_BBLEND) {
        int64_t below = b->sp > 0 ? b->clipanc[b->sp - 1] : -1;
        b->stk[b->sp] = i;
        b->clipanc[b->sp] = (k == K_BCLIP) ? i : below;
        if (inset) {
            if (k == K_BCLIP)
                memcpy(b->reg + 4 * b->sp, inner, sizeof inner);
            else
                inset_region(b, b->reg + 4 * b->sp);
        }
        b->sp++;
    } else if (k == K_ECLIP || k == K_EBLEND) {
        b->sp--;
    }
}

static void b_close(builder *b) {
    int64_t o = b->stk[b->sp - 1];
    b_emit(b, b->kind[o] == K_BCLIP ? K_ECLIP : K_EBLEND);
}

/* One open, drawn clip or blend with equal probability. */
static void b_open_random(builder *b) { b_emit(b, rng_u01(&b->r) < 0.5 ? K_BCLIP : K_BBLEND); }

/*
 * Constrained random walk of exactly `len` elements that starts and ends at
 * the current depth (relative depth 0) and never exceeds relative depth `cap`.
 * At each step with r slots left and relative depth d:
 *   d == r                          -> close;
 *   u < 0.25, d < cap, d <= r - 2   -> open (clip or blend, 50/50);
 *   u < 0.5 and d > 0               -> close;
 *   otherwise                       -> leaf.
 * `hook_at` (sorted, length n_hooks) lists walk steps before which `hook` is
 * called; the hook must leave the depth unchanged.
 */
typedef void (*hook_fn)(builder *, void *);

static void b_walk(builder *b, int64_t len, int64_t cap, const int64_t *hook_at, int64_t n_hooks,
                   hook_fn hook, void *ctx) {
    int64_t base = b->sp, h = 0;
    for (int64_t i = 0; i < len; ++i) {
        while (h < n_hooks && hook_at[h] == i) {
            hook(b, ctx);
            ++h;
        }
        int64_t d = b->sp - base, r = len - i;
        if (d == r) {
            b_close(b);
            continue;
        }
        double u = rng_u01(&b->r);
        if (u < 0.25 && d < cap && d <= r - 2)
            b_open_random(b);
        else if (u < 0.5 && d > 0)
            b_close(b);
        else
            b_emit(b, K_LEAF);
    }
    while (h < n_hooks) {
        hook(b, ctx);
        ++h;
    }
}

/* A nested chain: `depth` opens alternating BEGIN_CLIP / BEGIN_BLEND (clip
   first), `leaves` leaves at the bottom, then the matching closes. */
typedef struct { int64_t depth, leaves; } chain_ctx;

static void chain_hook(builder *b, void *vctx) {
    chain_ctx *c = (chain_ctx *)vctx;
    b->in_chain = 1;
    b->chain_first = 1;
    for (int64_t j = 0; j < c->depth; ++j) b_emit(b, (j & 1) ? K_BBLEND : K_BCLIP);
    b->in_chain = 0;
    for (int64_t j = 0; j < c->leaves; ++j) b_emit(b, K_LEAF);
    for (int64_t j = 0; j < c->depth; ++j) b_close(b);
}

/* --------------------------------------------------------------- API */

/* Plain walk of n elements, depth cap `cap`, box mode 0/1/2.  Returns 0 on success. */
int tbg_walk(uint32_t *kind, float *box, int64_t n, int64_t cap, uint64_t seed, int box_mode) {
    builder b;
    if (b_init(&b, kind, box, n, cap, seed, box_mode)) return -1;
    b_walk(&b, n, cap, NULL, 0, NULL, NULL);
    int ok = (b.pos == n && b.sp == 0);
    b_free(&b);
    return ok ? 0 : -2;
}

/* A walk of n_walk elements (cap `cap`) with `n_chains` nested chains of the
   given depth (and `leaves` leaves each) inserted before seeded walk steps.
   Total length n_walk + n_chains * (2*depth + leaves). */
int tbg_walk_with_chains(uint32_t *kind, float *box, int64_t n_walk, int64_t cap,
                         int64_t n_chains, int64_t depth, int64_t leaves, uint64_t seed,
                         int box_mode) {
    int64_t n = n_walk + n_chains * (2 * depth + leaves);
    builder b;
    if (b_init(&b, kind, box, n, cap + depth, seed, box_mode)) return -1;
    int64_t *at = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_chains > 0 ? n_chains : 1));
    if (!at) return -1;
    rng_t pr;
    rng_seed(&pr, tbg_splitmix64(seed ^ 0xC4A1Full));
    for (int64_t j = 0; j < n_chains; ++j) at[j] = rng_int(&pr, 0, n_walk - 1);
    /* insertion sort: n_chains is small */
    for (int64_t j = 1; j < n_chains; ++j) {
        int64_t v = at[j], k = j - 1;
        while (k >= 0 && at[k] > v) {
            at[k + 1] = at[k];
            --k;
        }
        at[k + 1] = v;
    }
    chain_ctx cc = {depth, leaves};
    b_walk(&b, n_walk, cap, at, n_chains, chain_hook, &cc);
    int ok = (b.pos == n && b.sp == 0);
    free(at);
    b_free(&b);
    return ok ? 0 : -2;
}

/* A chain of `depth` opens (alternating clip/blend) enclosing a walk of
   n_walk elements (cap `cap` above the chain), then `depth` closes. */
int tbg_chain_around_walk(uint32_t *kind, float *box, int64_t depth, int64_t n_walk, int64_t cap,
                          uint64_t seed, int box_mode) {
    int64_t n = 2 * depth + n_walk;
    builder b;
    if (b_init(&b, kind, box, n, depth + cap, seed, box_mode)) return -1;
    b.in_chain = 1;
    b.chain_first = 1;
    for (int64_t j = 0; j < depth; ++j) b_emit(&b, (j & 1) ? K_BBLEND : K_BCLIP);
    b.in_chain = 0;
    b_walk(&b, n_walk, cap, NULL, 0, NULL, NULL);
    for (int64_t j = 0; j < depth; ++j) b_close(&b);
    int ok = (b.pos == n && b.sp == 0);
    b_free(&b);
    return ok ? 0 : -2;
}

/* Ragged batch: scene sizes floor(2^U[lg_lo, lg_hi]) and depth caps U{cap_lo..cap_hi},
   each scene with its own seed splitmix64(seed ^ s).  Pass kind == NULL to only
   compute offsets (offsets has num_scenes + 1 entries).  Returns total length. */
int64_t tbg_batch(uint32_t *kind, float *box, int64_t *offsets, int64_t num_scenes, double lg_lo,
                  double lg_hi, int64_t cap_lo, int64_t cap_hi, uint64_t seed, int box_mode) {
    rng_t pr;
    rng_seed(&pr, seed);
    int64_t total = 0;
    int64_t *caps = (int64_t *)malloc(sizeof(int64_t) * (size_t)(num_scenes > 0 ? num_scenes : 1));
    if (!caps) return -1;
    offsets[0] = 0;
    for (int64_t s = 0; s < num_scenes; ++s) {
        double lg = lg_lo + rng_u01(&pr) * (lg_hi - lg_lo);
        int64_t sz = (int64_t)floor(pow(2.0, lg));
        caps[s] = rng_int(&pr, cap_lo, cap_hi);
        total += sz;
        offsets[s + 1] = total;
    }
    if (kind) {
        for (int64_t s = 0; s < num_scenes; ++s) {
            int64_t o = offsets[s], sz = offsets[s + 1] - o;
            if (tbg_walk(kind + o, box + 4 * o, sz, caps[s], tbg_splitmix64(seed ^ (uint64_t)s),
                         box_mode)) {
                free(caps);
                return -2;
            }
        }
    }
    free(caps);
    return total;
}

/* fp32 N(0,1) values by Box-Muller in double, rounded to fp32. */
void tbg_normal(float *out, int64_t n, uint64_t seed) {
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; i += 2) {
        double u1 = rng_u01(&r), u2 = rng_u01(&r);
        double rad = sqrt(-2.0 * log(1.0 - u1));
        out[i] = (float)(rad * cos(2.0 * M_PI * u2));
        if (i + 1 < n) out[i + 1] = (float)(rad * sin(2.0 * M_PI * u2));
    }
}

/* Raw stream of uniform u64 draws (exposed so tests can pin the generator). */
void tbg_raw(uint64_t *out, int64_t n, uint64_t seed) {
    rng_t r;
    rng_seed(&r, seed);
    for (int64_t i = 0; i < n; ++i) out[i] = rng_next(&r);
}

/* Typed bracket tokens for the parsing workload: the walk rule of tbg_walk
 * (depth cap `cap`), each open of a type drawn uniformly from [0, ntypes)
 * and written 2t+1, its close written 2t+2, every other step token 0.  With
 * probability p_bad a close is written with a different type (ntypes >= 2),
 * so the input is well nested but mistyped there.  Returns 0 on success. */
int tbg_brackets(uint32_t *tok, int64_t n, int64_t cap, uint32_t ntypes, double p_bad, uint64_t seed) {
    if (ntypes < 1) return -1;
    rng_t r;
    rng_seed(&r, seed);
    uint32_t *stk = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cap + 2));
    if (!stk) return -1;
    int64_t d = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t left = n - i;
        int what = 0; /* 0 none, 1 open, 2 close */
        if (d == left) {
            what = 2;
        } else {
            const double u = rng_u01(&r);
            if (u < 0.25 && d < cap && d <= left - 2)
                what = 1;
            else if (u < 0.5 && d > 0)
                what = 2;
        }
        if (what == 1) {
            const uint32_t t = (uint32_t)rng_int(&r, 0, (int64_t)ntypes - 1);
            stk[d++] = t;
            tok[i] = 2u * t + 1u;
        } else if (what == 2) {
            uint32_t t = stk[--d];
            if (ntypes >= 2 && rng_u01(&r) < p_bad) t = (t + 1 + (uint32_t)rng_int(&r, 0, ntypes - 2)) % ntypes;
            tok[i] = 2u * t + 2u;
        } else {
            tok[i] = 0u;
        }
    }
    free(stk);
    return d == 0 ? 0 : -2;
}

/* A draw-object stream around a tree: the m tree elements (kind, box) keep
 * their order and land on m of the n stream positions, each m-subset of
 * positions equally likely (selection sampling, Knuth TAOCP vol. 2,
 * Algorithm 3.4.2 S).  Every other position gets tag `other` and a box drawn
 * uniformly in [-1000, 1000)^4 (finite, not ordered), which a consumer must
 * ignore.  Returns 0, or -1 if m > n. */
int tbg_interleave(const uint32_t *kind, const float *box, int64_t m, int64_t n, uint32_t other,
                   uint64_t seed, uint32_t *tag_out, float *box_out) {
    if (m < 0 || m > n) return -1;
    rng_t r;
    rng_seed(&r, seed);
    int64_t need = m, j = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t left = n - i;
        const int take = need > 0 && (double)left * rng_u01(&r) < (double)need;
        if (take) {
            tag_out[i] = kind[j];
            memcpy(box_out + 4 * i, box + 4 * j, 4 * sizeof(float));
            ++j;
            --need;
        } else {
            tag_out[i] = other;
            for (int c = 0; c < 4; ++c) box_out[4 * i + c] = (float)(2000.0 * rng_u01(&r) - 1000.0);
        }
    }
    return 0;
}
