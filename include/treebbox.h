/*
 * libtreebbox -- bounding boxes on flattened scene trees, on AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * The operations follow R. Levien, "Fast GPU bounding boxes on
 * tree-structured scenes" (arXiv 2205.11659):
 *
 *  - A scene tree is flattened: a node with children is an open element,
 *    the encoding of its children, then a close element (Introduction,
 *    "Motivation").  Element kinds are tb_kind below.
 *  - Matching (section "The parentheses matching problem", Fig. 1): for
 *    every element, the index on top of the sequential stack before it is
 *    processed (`pm`; -1 at the root), and the classical partner of every
 *    open and close (`match`; -1 for leaves), which that section says is
 *    reconstructed from the former.
 *  - Boxes (Introduction; section "Parallel bounding boxes"): a leaf's box is
 *    its own box intersected with every clip node on its path to the root; a
 *    clip node's box is likewise its own box intersected with its clip
 *    ancestors; a blend node's box is the union of the clipped boxes of all
 *    leaves in the slice between its open and its close.  The node box is
 *    written at both the open and the close element (section "GPU
 *    implementation of clipping and blending", last paragraph).
 *
 * Conventions where the paper is silent:
 *  - tb_box is (x0, y0, x1, y1), fp32.  A box is non-empty iff x0 < x1 and
 *    y0 < y1; every empty result is written as EMPTY = (+inf, +inf, -inf,
 *    -inf).  Inputs must be NaN-free and hold no -0.0.
 *  - Blend nodes pass their enclosing clip context through unchanged; only
 *    leaves enter unions.  The box rows of END_CLIP, BEGIN_BLEND and
 *    END_BLEND inputs are ignored.
 *  - Results are bit-identical to the sequential walk: matching is integer
 *    work and fp32 max/min never rounds.
 *
 * Memory: every array pointer is a DEVICE pointer owned by the caller.  The
 * library never allocates; the caller passes a device workspace of at least
 * tb_workspace_bytes() bytes (contents need not be initialised; the library
 * overwrites what it reads).  Inputs are read-only; outputs must not alias
 * inputs or the workspace.  kind and index arrays must be 4-byte aligned,
 * box arrays 16-byte aligned, the workspace 256-byte aligned.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 * enqueue work on it and return without synchronising.  Two calls that
 * share a workspace must be ordered on one stream.
 *
 * Errors: the return value reports argument errors found on the host before
 * any work is enqueued (then nothing is enqueued), or TB_ERR_HIP if a launch
 * fails.  Errors in the data itself are OR-ed as TB_DATA_* bits into the
 * caller's device status word(s), which the call first clears; when a status
 * word is non-zero the outputs it covers are unspecified.
 */
#ifndef TREEBBOX_H
#define TREEBBOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TB_LEAF = 0,
    TB_BEGIN_CLIP = 1,
    TB_END_CLIP = 2,
    TB_BEGIN_BLEND = 3,
    TB_END_BLEND = 4,
    TB_OTHER = 5 /* tb_bbox_stream only: a stream element outside the tree */
} tb_kind;

typedef struct {
    float x0, y0, x1, y1;
} tb_box;

/* 2-D affine transform [a b c; d e f] on integer coordinates (x, y) ->
   (a x + b y + c, d x + e y + f), arithmetic modulo 2^32.  24 bytes. */
typedef struct {
    uint32_t a, b, c, d, e, f;
} tb_affine;

typedef enum {
    TB_OK = 0,
    TB_ERR_NULL = 1,      /* a required pointer is NULL */
    TB_ERR_SIZE = 2,      /* n < 0, n >= 2^31, num_scenes < 1, or sizes disagree */
    TB_ERR_ALIGN = 3,     /* a pointer violates the alignment stated above */
    TB_ERR_WORKSPACE = 4, /* ws_bytes < tb_workspace_bytes(...) */
    TB_ERR_ARG = 5,       /* any other invalid argument */
    TB_ERR_HIP = 6,       /* a HIP launch failed */
    TB_ERR_TOO_LARGE = 7  /* tb_bbox_noalloc: n above TB_NOALLOC_MAX_N */
} tb_status;

/* Device-side data error bits (OR-ed into the status word). */
#define TB_DATA_BAD_KIND 0x1u      /* a kind value above 4 */
#define TB_DATA_UNBALANCED 0x2u    /* a close with no open, or an open never closed */
#define TB_DATA_KIND_MISMATCH 0x4u /* END_CLIP closing BEGIN_BLEND or vice versa */
#define TB_DATA_BAD_OFFSETS 0x8u   /* batched: offsets not 0 = o[0] <= ... <= o[S] = total_n */
#define TB_DATA_GRAD_RANGE 0x10u   /* backward: a routed upstream gradient with |g| >= 2^31 or NaN */

/* Operation codes for tb_workspace_bytes. */
#define TB_OP_MATCH 0
#define TB_OP_BBOX 1
#define TB_OP_BBOX_BACKWARD 2
#define TB_OP_BBOX_BATCHED 3
#define TB_OP_COMPOSE 4
#define TB_OP_BBOX_STREAM 5
#define TB_OP_COMPOSE_F32 6
#define TB_OP_REDUCE_UP_F32 7

/* Workspace bytes needed by `op` for n elements (num_scenes is used by
   TB_OP_BBOX_BATCHED only; pass 1 otherwise).  Returns 0 for invalid sizes. */
size_t tb_workspace_bytes(int op, int64_t n, int64_t num_scenes);

/*
 * Parentheses matching over element kinds (section "The parentheses matching
 * problem"; the stronger output of Fig. 1 is `pm`).
 *   kind   [n]  uint32 tb_kind values                                 (in)
 *   match  [n]  int32 partner index, -1 for LEAF                      (out)
 *   pm     [n]  int32 top of the stack before element i, -1 = root    (out, nullable)
 *   dev_status [1] uint32                                             (out)
 * n == 0 is valid and enqueues only the status clear.
 */
tb_status tb_match(const uint32_t *kind, int64_t n, int32_t *match, int32_t *pm, void *ws,
                   size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * Matching over typed brackets, the primitive parsers need (section "The
 * parentheses matching problem" with several kinds of parentheses; the
 * paper names parsing among the method's applications).  Token 0 is no
 * bracket, 2t+1 opens a bracket of type t, 2t+2 closes one (so tokens 0..4
 * are the five element kinds, clip and blend being types 0 and 1).  Every
 * uint32 is a valid token.  Outputs as for tb_match; a close whose type
 * differs from its open's still matches it and sets
 * TB_DATA_KIND_MISMATCH; an unmatched close or open sets
 * TB_DATA_UNBALANCED.  Workspace: tb_workspace_bytes(TB_OP_MATCH, n, 1).
 *   tok    [n]  uint32 tokens                                       (in)
 *   match  [n]  int32 partner index, -1 for token 0                 (out)
 *   pm     [n]  int32 top of the stack before element i, -1 = root (out, nullable)
 *   dev_status [1] uint32                                           (out)
 */
tb_status tb_match_brackets(const uint32_t *tok, int64_t n, int32_t *match, int32_t *pm, void *ws,
                            size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * Matching plus node boxes: clip intersections down the tree and blend
 * unions up the tree (Introduction; sections "Parallel bounding boxes" and
 * "GPU implementation of clipping and blending").
 *   kind    [n]  uint32                                      (in)
 *   box_in  [n]  tb_box; rows of LEAF and BEGIN_CLIP used    (in)
 *   match   [n]  int32 partner, -1 for LEAF                  (out, nullable)
 *   box_out [n]  tb_box node box per element                 (out)
 *   dev_status [1] uint32                                    (out)
 */
tb_status tb_bbox(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                  tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                  void *stream);

/*
 * tb_bbox without a workspace argument, for callers that cannot allocate one
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same results as tb_bbox, bit for bit.  Intermediates live in
 * a fixed 64 MiB device array inside the library, one per GPU, held until
 * the process ends; nothing is allocated by the call.  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU race: order them
 * on one stream.  n <= TB_NOALLOC_MAX_N (2^20), else TB_ERR_TOO_LARGE before
 * any work is enqueued.  The array of the stream's device is used (the
 * current device for the NULL stream).
 *   kind, box_in, match, box_out, dev_status  as for tb_bbox
 */
#define TB_NOALLOC_MAX_N (1 << 20)
tb_status tb_bbox_noalloc(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                          tb_box *box_out, uint32_t *dev_status, void *stream);

/*
 * Gradient of tb_bbox's box_out with respect to box_in (not in the paper).
 * Each output coordinate of a non-EMPTY row routes its gradient to the one
 * input coordinate that attains it: for LEAF / BEGIN_CLIP / END_CLIP rows,
 * the lowest element index among the row's own box (END_CLIP: its BEGIN_CLIP)
 * and its enclosing BEGIN_CLIPs whose coordinate equals the output; for
 * blend rows, the lowest such index over the descendant leaves whose
 * non-EMPTY output equals the blend's coordinate.  Contributions are summed
 * exactly as 64-bit integers on a 2^-32 grid (each g rounded half-to-even to
 * the grid) and rounded once to fp32, so the result does not depend on
 * summation order.  Rounding to the grid makes a contribution with
 * |g| < 2^-9 inexact and one with |g| <= 2^-33 zero.  A routed g with
 * |g| >= 2^31 (or NaN) sets TB_DATA_GRAD_RANGE.  The integer sums wrap
 * modulo 2^64; precondition: each final sum fits in an int64 (the exact
 * gradient is below 2^31 in magnitude).
 * The forward's match output is not an argument: the pass recomputes the
 * pairs together with the attaining indices.
 *   kind, box_in [n]  as for tb_bbox                         (in)
 *   grad_out     [n]  tb_box upstream gradient               (in)
 *   grad_in      [n]  tb_box gradient w.r.t. box_in          (out)
 *   dev_status   [1]                                         (out)
 */
tb_status tb_bbox_backward(const uint32_t *kind, const tb_box *box_in, const tb_box *grad_out,
                           int64_t n, tb_box *grad_in, void *ws, size_t ws_bytes,
                           uint32_t *dev_status, void *stream);

/*
 * Many independent scenes in one call.  Scene s occupies elements
 * [offsets[s], offsets[s+1]) of the concatenated arrays; matching, clips and
 * unions never cross a scene boundary, and match indices are scene-local, so
 * each scene's rows are byte-identical to a tb_bbox call on that scene alone.
 *   offsets    [num_scenes+1] int64, device, 0 = o[0] <= ... <= o[S] = total_n (in)
 *   dev_status [num_scenes]   one status word per scene                       (out)
 * Other arguments as for tb_bbox, with n = total_n.
 */
tb_status tb_bbox_batched(const uint32_t *kind, const tb_box *box_in, const int64_t *offsets,
                          int64_t num_scenes, int64_t total_n, int32_t *match, tb_box *box_out,
                          void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * Composition of transforms down the tree: the same method applied to a
 * general, non-commutative monoid (the Introduction names transforms composed
 * down a skeleton as such an application).  Every open element, of either
 * kind, carries a transform; element i's output is the product of the
 * transforms of all opens enclosing it, outermost first (p.q applies q
 * first), including its own if it is an open; a close's output is its open's.
 * Arithmetic modulo 2^32 is exact and associative, so the result is the
 * sequential walk's bit for bit however the parallel steps group products.
 *   kind   [n]  uint32 tb_kind values; kind pairs are not checked   (in)
 *   xf_in  [n]  tb_affine, rows of opens used, 8-byte aligned        (in)
 *   xf_out [n]  tb_affine composed transform per element, 8-byte aligned (out)
 *   dev_status [1] uint32: TB_DATA_BAD_KIND, TB_DATA_UNBALANCED       (out)
 * Workspace: tb_workspace_bytes(TB_OP_COMPOSE, n, 1).
 */
tb_status tb_compose(const uint32_t *kind, const tb_affine *xf_in, int64_t n, tb_affine *xf_out,
                     void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * Composition of fp32 transforms down the tree: a monoid whose products
 * round, so the combine order is part of the result.  The order is that of
 * pointer jumping over the opens (section "Parallel bounding boxes", Clips):
 * every open starts with its own transform and a pointer to its enclosing
 * open; in each round all opens at once replace their value v by (value at
 * the pointer) . v and their pointer by the pointer's pointer, from the
 * previous round's values, until no pointer is left.  A leaf takes the value
 * of the open enclosing it (the identity at the root), a close that of its
 * open.  p . q applies q first; every product and every sum is one fp32
 * operation rounded to nearest even, no fused multiply-add:
 *   a = p.a*q.a + p.b*q.d,  b = p.a*q.b + p.b*q.e,  c = (p.a*q.c + p.b*q.f) + p.c,
 *   d = p.d*q.a + p.e*q.d,  e = p.d*q.b + p.e*q.e,  f = (p.d*q.c + p.e*q.f) + p.f.
 * Rounds cost a pass over all elements each; ceil(log2(depth + 1)) of them
 * do work (later launches return at once).
 *   kind   [n]  uint32 tb_kind values                                  (in)
 *   xf_in  [n]  6 floats [a b c d e f] per row, rows of opens used, 8-byte aligned (in)
 *   xf_out [n]  6 floats, the composed transform per element          (out)
 *   dev_status [1] uint32: as tb_match                                  (out)
 * Workspace: tb_workspace_bytes(TB_OP_COMPOSE_F32, n, 1).
 */
tb_status tb_compose_f32(const uint32_t *kind, const float *xf_in, int64_t n, float *xf_out, void *ws,
                         size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * The other direction with a rounding monoid: the fp32 transforms of the
 * leaves multiplied UP the tree (the Introduction states the method for
 * general monoids; blend unions are the paper's case going up).  An open
 * and its close get the ordered product of the transforms of the leaves
 * strictly between them, the leftmost leaf the leftmost factor (p . q as
 * in tb_compose_f32); an open with no leaf inside gets the identity; a leaf
 * gets its own transform.  The grouping is a segment tree over positions:
 * with N the smallest power of two >= n, leaf node N+i holds element i's
 * transform if it is a leaf, node v = node 2v . node 2v+1 (a side with no
 * leaf leaves the other unchanged), and the range of leaves is read
 * bottom-up (l = lo+N, r = hi+N+1; while l < r: if l odd L = L . node[l++];
 * if r odd R = node[--r] . R; l /= 2; r /= 2), result L . R.  Inputs must be
 * finite.  Rows of leaf inputs are used.
 *   kind, xf_in, xf_out, dev_status: as tb_compose_f32
 * Workspace: tb_workspace_bytes(TB_OP_REDUCE_UP_F32, n, 1) (48 B per
 * element of 2N tree nodes, plus matching).
 */
tb_status tb_reduce_up_f32(const uint32_t *kind, const float *xf_in, int64_t n, float *xf_out, void *ws,
                           size_t ws_bytes, uint32_t *dev_status, void *stream);

/*
 * Node boxes over a draw-object stream (Introduction: a renderer extracts
 * just the tree's elements from its scene description by stream compaction,
 * a prefix-sum application, and runs the algorithm on those only).  The
 * stream holds the tree's elements (tags TB_LEAF .. TB_END_BLEND, leaves
 * included since they enter blend unions) among elements outside the tree
 * (TB_OTHER).  The result is tb_bbox on the tree elements in stream order,
 * written back at their stream positions, with partners given as stream
 * positions.  Rows and match entries at TB_OTHER positions are not written.
 * A tag above TB_OTHER sets TB_DATA_BAD_KIND and is otherwise dropped like
 * TB_OTHER.  The extraction happens on the device: no host synchronisation.
 *   tag     [n]  uint32 tb_kind values, TB_OTHER allowed             (in)
 *   box_in  [n]  tb_box; rows of LEAF and BEGIN_CLIP used            (in)
 *   match   [n]  int32 partner stream position, -1 for LEAF         (out, nullable)
 *   box_out [n]  tb_box node box per tree element                    (out)
 *   dev_status [1] uint32                                            (out)
 * Workspace: tb_workspace_bytes(TB_OP_BBOX_STREAM, n, 1) (sized for every
 * element being a tree element).
 */
tb_status tb_bbox_stream(const uint32_t *tag, const tb_box *box_in, int64_t n, int32_t *match,
                         tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                         void *stream);

/*
 * Autotuning.  The paper finds that the best number of elements per thread
 * depends on the problem size (section "Performance results").  A call's
 * launch variant is: elements per thread of the main pass and of the
 * reduce pass (4 or 8 each; the partition stays 1024 elements, so the
 * workspace does not change) and close records per thread of the
 * cross-partition pass (2, 4 or 8; matching alone uses 4).  Results never
 * depend on the variant.  Calls of tb_match, tb_bbox and tb_bbox_batched
 * use, for their size class ceil(log2 n), the variant chosen for the
 * current device kind (architecture and compute-unit count), else the
 * default (4, 4, 4 for boxes; 8, 8, 4 for matching alone).  Matching with
 * parents (pm non-NULL) runs 4 elements per thread in the main pass whatever
 * the variant (8 is slower there).
 *
 * tb_tune_*: same arguments as the call they tune, plus `reps`; each
 * candidate variant runs one warm-up and `reps` timed calls on the caller's
 * input (outputs overwritten), the fastest median is kept for n's size
 * class, and the outputs are left as the chosen variant wrote them.  They
 * synchronise `stream` and create two HIP events.  Optional outputs:
 * *chosen, and ms[0], ms[1] = the chosen and the default variant's median
 * milliseconds.  Not for use under graph capture.
 */
typedef struct {
    int32_t resolve_elems; /* elements per thread of the main pass: 4 or 8 */
    int32_t reduce_elems;  /* elements per thread of the reduce pass: 4 or 8 */
    int32_t cross_records; /* close records per thread of the cross-partition pass: 2, 4, 8 */
} tb_variant;

tb_status tb_tune_match(const uint32_t *kind, int64_t n, int32_t *match, int32_t *pm, void *ws,
                        size_t ws_bytes, uint32_t *dev_status, void *stream, int reps,
                        tb_variant *chosen, float *ms);
tb_status tb_tune_bbox(const uint32_t *kind, const tb_box *box_in, int64_t n, int32_t *match,
                       tb_box *box_out, void *ws, size_t ws_bytes, uint32_t *dev_status,
                       void *stream, int reps, tb_variant *chosen, float *ms);
tb_status tb_tune_bbox_batched(const uint32_t *kind, const tb_box *box_in, const int64_t *offsets,
                               int64_t num_scenes, int64_t total_n, int32_t *match, tb_box *box_out,
                               void *ws, size_t ws_bytes, uint32_t *dev_status, void *stream,
                               int reps, tb_variant *chosen, float *ms);
/* The variant calls of `op` (TB_OP_MATCH, TB_OP_BBOX, TB_OP_BBOX_BATCHED)
   on n elements use on the current device; set pins one (NULL: back to the
   default; TB_ERR_ARG for an invalid variant or op). */
tb_status tb_variant_get(int op, int64_t n, tb_variant *out);
tb_status tb_variant_set(int op, int64_t n, const tb_variant *v);
/* The table of chosen variants as text (one line per device kind, op and
   size class); load merges a saved table (TB_ERR_ARG if the file cannot be
   read or is not such a table); clear forgets every choice. */
tb_status tb_tune_save(const char *path);
tb_status tb_tune_load(const char *path);
void tb_tune_clear(void);

/*
 * Profiling hook: when both are non-NULL, later calls record `before` and
 * `after` (hipEvent_t handles created by the caller) on the call's stream
 * immediately around the launch of the main per-partition kernel, so its
 * duration can be read with hipEventElapsedTime.  Pass NULLs to stop.  Not
 * thread-safe; meant for benchmarks.
 */
void tb_profile_events(void *before, void *after);

/* Static string naming a tb_status value. */
const char *tb_status_str(tb_status s);

#ifdef __cplusplus
}
#endif

#endif /* TREEBBOX_H */
