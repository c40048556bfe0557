/*
 * dt.h -- exact 3D Delaunay tetrahedralization on one AMD MI355X (gfx950).
 *
 * The library builds the Delaunay tetrahedralization of fp64 point sets by incremental
 * Bowyer-Watson insertion (the "Delaunay kernel" DT <- DT - C(DT, p) + B(DT, p) of
 * Marot, Pellerin and Remacle, "One machine, one minute, three billion tetrahedra",
 * Sec. 2.1, Eq. (1) and Algorithm 1), with thousands of insertions per round on the GPU.
 *
 * Problem (Sec. 1): given n points S, the output tetrahedra have pairwise disjoint
 * interiors and their union is the convex hull of S; every distinct point of S is a
 * vertex, and no point of S lies strictly inside any output circumsphere.  Points in
 * non-general position are resolved by symbolic perturbation (Sec. 2.4, item 3): the
 * lifted coordinate |p_i|^2 of the point with input index i is perturbed by eps^delta_i,
 * delta strictly decreasing in i.  The result is therefore unique and does not depend on
 * the insertion order, the round packing or the launch configuration.
 *
 * Conventions (Sec. 2.2): a tetrahedron (v0,v1,v2,v3) has orient3d(v0,v1,v2,v3) > 0 with
 * orient3d(a,b,c,d) = (b-a).((c-a)x(d-a)); facet j is the facet opposite vertex vj.
 *
 * Memory: every pointer argument may be host memory or device memory of the context's
 * device (the library checks with hipPointerGetAttributes).  The caller owns all buffers
 * it passes; the library copies what it needs and never keeps a caller pointer.  All work
 * runs on the context's stream; every call returns after the work has completed.
 * A context is not thread-safe: use one context per host thread.
 *
 * Errors: every function returns DT_OK or one of the DT_E_* codes below and never
 * throws across the ABI; dt_last_error() gives a readable message for the last failure.
 */
#ifndef DT_H
#define DT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DT_OK = 0,
    DT_E_ARG = 1,        /* NULL pointer, bad size or bad option                        */
    DT_E_INPUT = 2,      /* a coordinate is not finite or has magnitude outside the
                            accepted range (0, or |x| in [2^-120, 2^120))                 */
    DT_E_DEGENERATE = 3, /* fewer than four affinely independent distinct points        */
    DT_E_CAPACITY = 4,   /* device memory exhausted or a size limit exceeded            */
    DT_E_INCOMPLETE = 5, /* the round limit (dt_options.max_rounds) was reached         */
    DT_E_DEVICE = 6,     /* a HIP runtime call failed                                   */
    DT_E_INTERNAL = 7    /* an internal consistency check failed (a bug)                */
};

typedef struct dt_ctx dt_ctx;

typedef struct {
    int device;             /* HIP device ordinal                                        */
    void *stream;           /* hipStream_t to run on; NULL: the library creates one       */
    uint32_t round_size;    /* most insertions attempted per round; 0: automatic         */
    uint32_t cavity_cap;    /* cavity tetrahedra buffered per insertion; 0: automatic     */
    uint64_t capacity_tets; /* initial tetrahedron pool (grown on demand); 0: automatic   */
    uint64_t seed;          /* seed of the randomized insertion levels (BRIO, Sec. 2.3)  */
    uint32_t max_rounds;    /* 0: unlimited; otherwise DT_E_INCOMPLETE beyond it          */
    int timing;             /* 1: time the two insertion kernels of every round with HIP
                               events (three per round); 2: the cavity kernel of rounds of
                               at least 32768 candidates only (two per such round: an
                               event record leaves the GPU idle for a few microseconds,
                               which short rounds feel most)                             */
    double round_fraction;  /* round size as a fraction of the current vertex count;
                               0: automatic (1/16, and 3/32 for rounds that stay below
                               32768 candidates)                                         */
    uint32_t lanes_per_insert; /* lanes of a wavefront cooperating on one insertion in the
                                  walk and cavity search: 4, 8, 16, 32 or 64 in every
                                  round; 0: automatic (64 in rounds of fewer than 32768
                                  candidates, whose time is their slowest insertion's,
                                  16 in larger ones)                                     */
    int scheduler;          /* DT_SCHED_PLAIN (0) or DT_SCHED_LEARNED (1: uses the model of
                               dt_load_model or dt_train_model; without one the call runs
                               the plain order and counts dt_stats.sched_fallbacks)      */
    int log_points;         /* 1: record the attempts of every point (dt_get_point_log)  */
    int index_bits;         /* width of the adjacency codes 4 t + f (Sec. 2.2): 32 (pools
                               up to 2^30 - 1 tetrahedron slots), 64 (up to 2^32 - 16
                               slots, the same 64-byte records), or 0: 32 while the pool
                               fits, widened to 64 when it must grow past that           */
    int adaptive_curve;     /* 0: the Moore curve on the grid of level ceil(log2(n) / 3)
                               (Sec. 2.3); 1: on the deepest grid the sort key holds (21
                               levels for one cloud), which orders the points of a crowded
                               cell by the curve's finer levels, an adaptive curve for
                               non-uniform inputs (the Conclusion's open point).  The
                               triangulation is the same either way.                     */
    int subdet_cache;       /* 1: keep four sub-determinants per tetrahedron and the
                               largest of its edge-vector coordinates (40 bytes) so that
                               the cavity search's insphere test is a dot product that
                               reads one vertex (Sec. 2.4); each new tetrahedron pays for
                               them in the DelaunayBall step.  Signs the cached filter
                               cannot decide go to the exact predicates; the result is the
                               same.                                                     */
    uint32_t walk_cap;      /* walk steps after which an attempt of a regular round stops;
                               its point retries in the next round, resuming the walk from
                               where it stopped (a launch then ends with its typical
                               attempts, not with one long walk).  0: automatic (16);
                               UINT32_MAX: no cap.  The result never depends on it.      */
    uint32_t large_lanes;   /* lanes per insertion in rounds for cavities beyond the
                               regular rounds' 128-entry buffers: 64 (one wavefront,
                               16 cavity tetrahedra per breadth-first step) or 256 (a
                               256-thread block, 64 per step); 0: automatic (256)        */
    int graph_rounds;       /* 1: launch each regular round (the candidate fill, both cavity
                               passes, the DelaunayBall kernel and the three round-end
                               kernels) as one HIP graph, built once per launch shape and
                               given each round's arguments and grids; rounds for large
                               cavities, timed rounds and traced rounds stay separate
                               launches.  0: separate launches.  The result is the same.  */
} dt_options;

enum { DT_SCHED_PLAIN = 0, DT_SCHED_LEARNED = 1 };

/* Counters of the work done since dt_create or the last dt_clear. */
typedef struct {
    uint64_t points;          /* points passed to dt_insert_points                     */
    uint64_t vertices;        /* distinct points in the triangulation                  */
    uint64_t duplicates;      /* exact duplicates dropped (lowest input index kept)    */
    uint64_t tets;            /* finite tetrahedra of the current triangulation        */
    uint64_t rounds;          /* insertion rounds                                      */
    uint64_t attempts;        /* insertion attempts (walk + cavity) over all rounds    */
    uint64_t inserted;        /* successful insertions                                 */
    uint64_t conflicts;       /* attempts that lost a claim to a lower-ranked insertion */
    uint64_t overflows;       /* attempts whose cavity outgrew the per-insertion buffer */
    uint64_t walk_steps;      /* tetrahedra crossed by point location                  */
    uint64_t cavity_tets;     /* tetrahedra deleted by successful insertions           */
    uint64_t boundary_facets; /* tetrahedra created by successful insertions           */
    uint64_t orient_calls, orient_exact;     /* orient3d evaluations / exact fallbacks  */
    uint64_t insphere_calls, insphere_exact; /* insphere evaluations / exact fallbacks  */
    uint64_t perturbed;       /* insphere decisions taken by the symbolic perturbation  */
    double ms_total;          /* wall time of dt_insert_points calls (host clock)      */
    double ms_sort;           /* validation, Moore keys, radix sort, dedupe, anchors   */
    double ms_insert;         /* all insertion rounds                                  */
    /* with dt_options.timing = 1: HIP-event time of the two insertion kernels */
    uint64_t cavity_launches, ball_launches;
    double ms_cavity_kernel, ms_ball_kernel;
    uint64_t cavity_units, ball_units; /* attempts processed / insertions completed   */
    uint64_t sched_fallbacks; /* calls with DT_SCHED_LEARNED but no model loaded, run in the
                                 plain order instead                                     */
    uint64_t index_bits;      /* adjacency code width of the current pool (0: no pool)   */
    uint64_t dropped_slots;   /* freed slots left unused because the free list was full  */
    uint64_t deferred;        /* attempts whose fp64 filter left a sign undecided, run
                                 again with exact predicates in the same round           */
    uint64_t walk_caps;       /* attempts stopped by dt_options.walk_cap (counted among
                                 the conflicts too: they retry in the next round)        */
    uint64_t timed_attempts, timed_insertions; /* attempts and insertions of the rounds
                                 timed by dt_options.timing (cavity_launches of them)    */
    uint64_t graph_rounds;    /* rounds launched as one HIP graph (dt_options.graph_rounds) */
} dt_stats;

/* Fill *opt with the defaults (device 0, library stream, automatic sizes, seed 0x5EED). */
void dt_default_options(dt_options *opt);

/* Create a context on opt->device (opt may be NULL for the defaults).
   *out receives the context; release it with dt_destroy. */
int dt_create(dt_ctx **out, const dt_options *opt);

/* Insert n points, xyz[3*i+0..2] = (x, y, z) of point i, fp64, array of structures,
   host or device memory.  Point i of this call gets the global input index
   (points inserted before) + i.  On return the context holds the Delaunay
   tetrahedralization of all points inserted so far (Algorithm 1 run as concurrent
   rounds).  An exact duplicate of an earlier point is not a vertex.  The first call
   must provide four affinely independent points or it fails with DT_E_DEGENERATE and
   leaves the context empty.  After DT_E_ARG, DT_E_INPUT or DT_E_DEGENERATE the context
   is as it was before the call; after DT_E_CAPACITY, DT_E_INCOMPLETE, DT_E_DEVICE or
   DT_E_INTERNAL only dt_clear, dt_get_stats, dt_last_error and dt_destroy are
   meaningful.  n = 0 does nothing and returns DT_OK.  Limits: fewer than 2^30 points per
   call and 2^31 in all (DT_E_CAPACITY); fewer than 2^30 tetrahedron slots with 32-bit
   adjacency codes, 2^32 - 16 with 64-bit codes (dt_options.index_bits). */
int dt_insert_points(dt_ctx *ctx, const double *xyz, uint64_t n);

/* Export the finite tetrahedra.  *num_tets is in/out: on input the capacity of the
   buffers in tetrahedra, on output the number T of tetrahedra (also when it exceeds the
   capacity, in which case nothing is written and DT_E_ARG is returned).  tets
   (4*T uint32, may be NULL) receives the global input indices of each tetrahedron's
   vertices in positive orientation; nbrs (4*T int64, may be NULL) receives, for facet j,
   the index of the tetrahedron across it or -1 on the convex hull.  Pass both NULL to
   query T.  Host or device pointers. */
int dt_get_tets(dt_ctx *ctx, uint32_t *tets, int64_t *nbrs, uint64_t *num_tets);

/* Triangulate num_clouds independent point clouds in one pass (the rounds of all clouds run
   in the same kernel launches).  Cloud k is xyz[3*offsets[k] .. 3*offsets[k+1]) (fp64 AoS,
   host or device memory); offsets (host memory, num_clouds + 1 entries, offsets[0] = 0,
   at least 4 points per cloud) are not retained.  Each cloud gets the Delaunay
   tetrahedralization of its own points (Algorithm 1), exactly as if it were inserted alone
   into a fresh context.  The context must be empty (new or after dt_clear), and
   dt_insert_points is refused until the next dt_clear, also after a call that fails past
   its argument checks (DT_E_ARG for NULL pointers, bad offsets or too few points in a cloud
   leaves the context untouched).  Errors as dt_insert_points; DT_E_DEGENERATE names the
   first degenerate cloud in dt_last_error.  Limits: fewer than 2^30 points in all, and the
   tetrahedron slots of dt_insert_points. */
int dt_insert_batch(dt_ctx *ctx, const double *xyz, const uint64_t *offsets, uint32_t num_clouds);

/* Export the finite tetrahedra of one cloud of the context (cloud 0 after dt_insert_points),
   with the same conventions as dt_get_tets but local to the cloud: vertex indices are
   input indices within the cloud (0 .. its size - 1), and neighbour indices refer to this
   call's output (-1 on the cloud's convex hull).  *num_tets is in/out as in dt_get_tets;
   pass both buffers NULL to query the count.  Host or device pointers. */
int dt_get_tets_batch(dt_ctx *ctx, uint32_t cloud, uint32_t *tets, int64_t *nbrs, uint64_t *num_tets);

/* Autotuner: triangulates the n sample points (host or device memory) once per launch
   configuration - lanes per insertion {automatic, 8, 16, 32}, round fraction {automatic, 3/64,
   3/32},
   cavity cap {64, 128}, lanes per insertion for large cavities {64, 256} (a wavefront or a
   256-thread block) - after one warm-up run, and keeps
   the fastest (host wall time of dt_insert_points) for the sample's size class,
   floor(log2 n).  Later insertions use the choice of the tuned class nearest to their own
   point count (ties to the larger class); with no class tuned, dt_options decide.  Tune at
   the size that will be run: choices do not carry over between sizes.  *best (may be NULL)
   receives the chosen options, *best_ms (may be NULL) its time.  The context must be empty
   and is empty again on return; the statistics are reset.  Results never depend on these
   options. */
int dt_autotune(dt_ctx *ctx, const double *xyz, uint64_t n, dt_options *best, double *best_ms);

/* Forgets every choice of dt_autotune; insertions use dt_options again. */
int dt_autotune_reset(dt_ctx *ctx);

/* ---- learned insertion scheduler (not in the paper; the output never depends on it) ----
   An MLP 16 -> 64 -> 64 -> 3 (BF16 weights, FP32 accumulation) maps features of each point
   (log distances to its curve neighbours and anchor, BRIO level, position in the box) to a
   cost (predicted log2(1 + attempts)) and two walk-start logits (curve neighbour / anchor).
   With dt_options.scheduler = DT_SCHED_LEARNED each BRIO level is inserted in two halves,
   the points predicted cheap (cost at most the median training cost) first, and the walk
   starts where the MLP predicts.  When the costly training points needed 3 attempts or
   more on average, rounds over the costly halves are half the usual size. */

/* After a dt_insert_points run with dt_options.log_points = 1: training samples of its
   points, in curve order - features (num_points x 16 fp32), cost target log2(1 + attempts)
   and bucket label (1 when the anchor is closer to the point than every curve neighbour
   within 4 records that belongs to a lower BRIO level, and at least one such neighbour
   exists; 0 otherwise).
   *num_points in/out as in dt_get_tets (NULL buffers: query).  Host or device pointers. */
int dt_get_point_log(dt_ctx *ctx, float *features, float *cost, uint8_t *bucket, uint64_t *num_points);

/* Train a model from scratch on n samples (host memory, as from dt_get_point_log): squared
   error on the cost plus softmax cross-entropy on the bucket, Adam (learning rate lr),
   minibatches of 4096 in a seeded random order, `epochs` passes, on the device.  The model
   (a header and the fp32 weights) is written to model (*model_bytes in/out; NULL model:
   query the size) and loaded into the context. */
int dt_train_model(dt_ctx *ctx, const float *features, const float *cost, const uint8_t *bucket, uint64_t n,
                   uint32_t epochs, float lr, uint64_t seed, void *model, size_t *model_bytes);

/* Load a model written by dt_train_model (host memory, not retained). */
int dt_load_model(dt_ctx *ctx, const void *model, size_t bytes);

/* Test hook: the loaded model's outputs (n x 3 fp32) for n feature rows (n x 16 fp32). */
int dt_debug_mlp(dt_ctx *ctx, const float *features, uint64_t n, float *out);

/* Test hook: gradient (NPARAM fp32, parameter order W1[16][64], b1, W2[64][64], b2,
   W3[64][3], b3) of the mean training loss of the loaded model over n samples, and *loss
   (may be NULL) = the summed per-sample loss.  Host or device pointers. */
int dt_debug_mlp_grad(dt_ctx *ctx, const float *features, const float *cost, const uint8_t *bucket, uint32_t n,
                      float *grad, float *loss);

/* ---- Delaunay refinement (Sec. 4) ----
   Refines the context's triangulation (built by dt_insert_points; not a batch) by inserting
   circumcentres, as the paper's mesh generator does with its size field, here one constant
   h.  Each step: every tetrahedron with squared circumradius above (1.4 h)^2 proposes its
   circumcentre (fp64, one fixed formula over its vertices in ascending input index, no
   fused operations); a proposal is a candidate only strictly inside the convex hull (exact
   orient3d against every hull facet), so the hull never changes; candidates are taken in
   the order of their Moore key in the grid of the points present when the call starts, then
   of their tetrahedron's sorted vertex indices, and one is kept iff no vertex and no kept
   earlier candidate lies closer than 0.7 h (squared distances in fp64); the kept points are
   inserted in that order (their input indices follow it).  Steps repeat until one keeps
   nothing, or max_steps.  step_counts (2 * max_steps uint32, may be NULL) receives each
   step's candidates and kept points; *num_steps and *inserted (may be NULL) the steps run
   and the points added.  h must be positive and finite and not below about 2^-20 of the
   point set's extent (DT_E_ARG).  Other errors as dt_insert_points. */
int dt_refine(dt_ctx *ctx, double h, uint32_t max_steps, uint32_t *step_counts, uint32_t *num_steps,
              uint64_t *inserted);

/* Coordinates of every point inserted so far, xyz[3*i..3*i+2] for global input index i (fp64,
   host or device memory); *num_points in/out as in dt_get_tets (NULL xyz: query).  Not for a
   batch of clouds. */
int dt_get_points(dt_ctx *ctx, double *xyz, uint64_t *num_points);

/* ---- triangulation without device allocation ----
   For callers that cannot allocate device memory: code under HIP graph capture, tight
   serving loops, harnesses that forbid hipMalloc.  Triangulates the n points at xyz (fp64
   AoS, host or device memory) on `device` and the given hipStream_t (NULL: the null
   stream), exactly as dt_create + dt_insert_points + dt_get_tets would (same unique
   result), and returns when done.  Every device buffer comes from a static array of
   DT_NOALLOC_SCRATCH_BYTES that each GPU the call runs on holds until the process ends; the
   call makes no hipMalloc, hipFree or other allocating call (the first call on a device only
   looks up the array's address).  The caller owns xyz and the outputs: tets (4*T uint32),
   nbrs (4*T int64), each may be NULL, host or device memory; *num_tets is in/out as in
   dt_get_tets (both NULL: the count only, after triangulating).  n above
   DT_NOALLOC_MAX_POINTS, or a result that does not fit the array, returns DT_E_CAPACITY;
   other errors as dt_insert_points.  Calls on one device share the array: calls that
   overlap on one device race.  No context, no statistics. */
#define DT_NOALLOC_MAX_POINTS 65536u
#define DT_NOALLOC_SCRATCH_BYTES (128u << 20)
int dt_triangulate_noalloc(int device, void *stream, const double *xyz, uint64_t n, uint32_t *tets,
                           int64_t *nbrs, uint64_t *num_tets);

/* Drop every point and tetrahedron but keep the device allocations. */
int dt_clear(dt_ctx *ctx);

/* Release the context and its device memory. */
int dt_destroy(dt_ctx *ctx);

/* Copy the counters into *out. */
int dt_get_stats(const dt_ctx *ctx, dt_stats *out);

/* Readable message of the last error on this context (never NULL). */
const char *dt_last_error(const dt_ctx *ctx);

/* ---- test hooks: the kernels of the hot path run on caller data ---- */

/* Sort step (Sec. 2.3): for n points (device or host xyz) computes the sort key
   (BRIO level << 3m | Moore index; the Moore index alone when 3m + 8 > 64, as with the
   adaptive curve) of every point and the stable sorted order.
   keys (n uint64) receives the keys in input order, perm (n uint32) the input index of
   the point at each sorted position; *moore_m receives m.  Device or host outputs. */
int dt_debug_sort(dt_ctx *ctx, const double *xyz, uint64_t n, uint64_t *keys, uint32_t *perm,
                  int *moore_m);

/* Sets the context's round counter (the stamp of the next round's claims).  Claim stamps
   take the low 32 bits of the counter; when they wrap, the library resets every claim word
   before the round.  Lets a test cross the wrap without 2^32 rounds. */
int dt_debug_set_round_counter(dt_ctx *ctx, uint64_t rounds);

/* With dt_options.index_bits = 0, a pool with 32-bit codes is widened to 64-bit codes when
   it must grow past `slots` (default and maximum 2^30 - 1; at least 4096) instead of past
   2^30 - 1: lets a test widen a pool in the middle of an insertion without 2^30 slots. */
int dt_debug_widen_at(dt_ctx *ctx, uint64_t slots);

/* Predicates (Sec. 2.4): for k records evaluates, per record r,
   kind 0: orient3d sign of pts[12r .. 12r+11] (four points);
   kind 1: insphere sign of the unperturbed lifted determinant of pts[15r ..] (five points);
   kind 2: sign of the perturbed lifted determinant, input indices idx[5r .. 5r+4].
   out[r] in {-1, 0, 1}.  Device or host buffers. */
int dt_debug_predicates(dt_ctx *ctx, int kind, const double *pts, const int64_t *idx,
                        uint64_t k, int8_t *out);

#ifdef __cplusplus
}
#endif
#endif
