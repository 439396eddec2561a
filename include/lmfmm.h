/*
 * lmfmm.h -- C ABI of the MI355X layered-media FMM for the reflected field g_2^t.
 *
 * The operator (Cho & Huang, arXiv 1902.08250, Section 1; Section 3 Example 4):
 *
 *   u_i = sum_j g_2^t(x_i, x_j) q_j,
 *   g_2^t(x1,y1; x0,y0) = Int_R e^{s2 y1 + i lam x1} e^{-s1 y0 - i lam x0} sigma_2^t(lam)/(4 pi s2) d lam,
 *   s_m = sqrt(lam^2 - k_m^2) (principal branch),
 *
 * for sources x_j in the top layer (y > 0) and targets x_i in the middle layer
 * (-d < y < 0) of a three-layer medium with wave numbers k1, k2, k3 (Im k >= 0)
 * and interfaces y = 0 and y = -d.  The apply is the adapted free-space FMM of
 * Section 2 (Algorithm 1): quadtree, source-to-multipole and multipole-to-
 * multipole with the free-space Helmholtz operators for k1, multipole-to-local
 * by Sommerfeld-integral translation matrices (Lemma M2L), local-to-local and
 * local evaluation with the free-space operators for k2, and the near field by
 * direct Sommerfeld quadrature on deformed contours (Section 4.2).  The
 * plan option "component" switches the same passes to the other three-layer
 * components g_2^b, g_1^s, g_3^s or to the impedance half-space (Section 3,
 * Examples 3 and 4).
 *
 * Conventions shared by every entry point:
 *   - All point and density arrays are DEVICE pointers owned by the caller and
 *     must stay valid until the work queued on the given stream completes.
 *   - Coordinates are float64, structure of arrays [2][n]: x[0..n), y[0..n).
 *   - Densities are interleaved complex, [nrhs][n]: complex128 (re, im float64)
 *     for LMFMM_C128, complex64 (re, im float32) for LMFMM_C64_MIXED.
 *   - stream is a hipStream_t (NULL = the default stream).  Entry points queue
 *     work asynchronously except where noted; argument errors are returned
 *     synchronously and nothing is queued.
 *   - A plan is not thread-safe; use one plan per host thread.
 *   - Status codes are returned, never thrown; lmfmm_last_error() gives the
 *     thread-local message of the last failure.
 */
#ifndef LMFMM_H
#define LMFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lmfmm_plan_s *lmfmm_plan;

enum {
    LMFMM_OK = 0,
    LMFMM_EINVAL = -1,  /* bad argument (null pointer, size, option)            */
    LMFMM_EDOMAIN = -2, /* a point lies outside its layer or is not finite      */
    LMFMM_ENOMEM = -3,  /* device or host allocation failed                     */
    LMFMM_EHIP = -4,    /* a HIP runtime call failed                            */
    LMFMM_ETOL = -5,    /* the requested tolerance cannot be met                */
    LMFMM_ENODEV = -6   /* no usable GPU                                        */
};

enum {
    LMFMM_C128 = 0,       /* FP64 throughout                                      */
    LMFMM_C64_MIXED = 1   /* FP32 expansions and translations; sigma, quadrature
                             weights and the near field stay FP64                */
};

/* Create a plan for the medium (Section 3 Example 4).
 *   k:     {Re k1, Im k1, Re k2, Im k2, Re k3, Im k3}, Re k > 0, Im k >= 0.
 *   d:     thickness of the middle layer, d > 0.
 *   order: expansion order p of the multipole/local series (truncation of
 *          the sums over p in Section 2), 1 <= order <= 256; the order used at
 *          a level is max(order, the order that tol requires there).
 *   tol:   target relative accuracy, 0 < tol < 1.
 * Queues the sigma_2^t quadrature tables on the null stream and synchronizes.
 * On success *out receives the plan (destroy with lmfmm_destroy). */
int lmfmm_create(const double k[6], double d, int order, double tol, lmfmm_plan *out);

/* Release a plan and its device memory (synchronizes the device). */
int lmfmm_destroy(lmfmm_plan plan);

/* Set an option (string key/value).  Keys:
 *   "levels"      quadtree depth L >= 1, or "auto" (default, ~40 points/leaf)
 *   "fixed_order" "1": use exactly `order` at every level, ignoring tol
 *   "domain"      "xmin,xmax,ys_max,yt_min": use this box in place of the
 *                 points' bounding box (x range of all points, largest
 *                 source y, smallest target y); skips the bounding-box
 *                 readback, so an apply queues no host synchronisation.
 *                 Points outside it raise the device error flag (see
 *                 lmfmm_sync_status).  "auto" (default) clears it.
 *   "kr_max"      largest k R (R = box half-diagonal, k = max |k1|, |k2|) of
 *                 a level that carries expansions (default 8): coarser
 *                 levels are skipped and the coarsest expansion level
 *                 translates between all its non-adjacent boxes
 *   "graph"       "1" (default): when two consecutive applies have the same
 *                 geometry, pointers, sizes and tables, the second captures
 *                 its launch sequence in a HIP graph and later ones replay it
 *                 (one launch).  Without a fixed domain the graph starts with
 *                 the bounding-box kernels: an apply with the same pointers,
 *                 sizes and options launches it before the box is known, and
 *                 computes again if the box turns out different from the one
 *                 the graph was captured for.  "0": always launch kernel by
 *                 kernel
 *   "near_sweep"  "1" (default): near field by x-ordered sweeps over the node
 *                 table; "0": the pairwise sum (same quadrature)
 *   "near"        "1" (default) / "0": include / skip the near field
 *   "far"         "1" (default) / "0": include / skip the far field
 *   "component"   the field component the plan applies (Section 3), sources
 *                 always in the top layer (y > 0):
 *                   "2t" (default) g_2^t, targets -d < y < 0;
 *                   "2b" g_2^b (Example 4), targets -d < y < 0;
 *                   "1s" g_1^s (Example 4), targets y > 0;
 *                   "3s" g_3^s (Example 4), targets y < -d;
 *                   "impedance" the reflected field of the impedance
 *                   half-space (Example 3) with wave number k1 (k2, k3 and
 *                   d unused), targets y > 0.
 *                 Each is applied by the same passes: targets enter the tree
 *                 at their image y' = -y (1s, impedance) or y' = -y - 2d
 *                 (2b), where the component's exponent becomes that of
 *                 g_2^t; the local expansions use the target layer's wave
 *                 number.  Setting it discards the plan's tables.
 *   "alpha"       impedance constant of the "impedance" component (default
 *                 0): the total field u satisfies u_y + i k1 alpha u = 0 on
 *                 y = 0 (density (s1 + i k1 alpha) / (s1 - i k1 alpha)).
 *                 Setting it discards the plan's tables.
 *   "tree_sort"   grouping of the points by leaf (Algorithm 1, Step 1):
 *                 "radix": a stable radix sort of the leaf keys (no atomics
 *                 per point); "count": a counting sort with one atomic per
 *                 point and a per-leaf sort of the original indices; "auto"
 *                 (default): radix from 3e5 points on (counted over all
 *                 instances of a batched apply).  Both give every leaf its
 *                 points in increasing original index, so the results are
 *                 the same bit for bit.
 *   "m2l_mfma"    "1": multipole-to-local as products of the class tables
 *                 with tiles of boxes x right-hand sides on the matrix cores;
 *                 "0": one matrix-vector product per box pair list; "auto"
 *                 (default): the matrix cores from 4 right-hand sides on
 *                 (FP32 expansions) or 3 (FP64), the vector form below
 *   "shift_mfma"  "1" (default): M2M and L2L as products of the shift tables
 *                 with tiles of boxes x right-hand sides on the matrix cores;
 *                 "0": one matrix-vector product per box
 *   "p2m_series"  "1" (default): P2M by the ascending series of J_q where the
 *                 leaves' k1 R <= 3 (for FP32 expansions only where leaves hold
 *                 40 points or more on average); "0": the recurrence form
 *                 everywhere
 *   "eval_levels" "1" (default): each leaf evaluates the local expansion of
 *                 the level where its far field is complete (its ancestor's),
 *                 and only the expansions read are shifted down; "0": every
 *                 leaf evaluates its own, shifted down level by level
 *   "timing"      "1": record a HIP event on the apply's stream before every
 *                 kernel (or group of tree-build kernels) of each apply and
 *                 accumulate the durations per kernel in
 *                 lmfmm_stats.kernel_ms; "0" stops; "reset" zeroes the sums
 * Returns LMFMM_EINVAL for an unknown key or malformed value. */
int lmfmm_set_option(lmfmm_plan plan, const char *key, const char *value);

/* Forward apply (Algorithm 1, Steps 1-4): u[r][i] = sum_j g_2^t(tgt_i, src_j) q[r][j].
 *   n_src, src_xy: source count and coordinates [2][n_src] (y > 0).
 *   q:     densities [nrhs][n_src].
 *   n_tgt, tgt_xy: target count and coordinates [2][n_tgt] (-d < y < 0; the
 *          layer of the plan's "component" otherwise).
 *   u:     output [nrhs][n_tgt], overwritten.
 *   nrhs:  number of right-hand sides, 1 <= nrhs <= 64.
 *   precision: LMFMM_C128 or LMFMM_C64_MIXED (selects the dtype of q and u).
 * Unless the "domain" option is set, the call waits for the points' bounding
 * box, which the device writes to host memory (the host spins on it, and after
 * 20 ms synchronises the stream).  Points outside their layer are reported as
 * LMFMM_EDOMAIN by the host check of that bounding box, or by
 * lmfmm_sync_status when a fixed domain is used. */
int lmfmm_apply(lmfmm_plan plan, int64_t n_src, const double *src_xy, const void *q, int64_t n_tgt,
                const double *tgt_xy, void *u, int nrhs, int precision, void *stream);

/* Size of the fixed device array that lmfmm_apply_noalloc works in. */
#define LMFMM_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* lmfmm_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and result as lmfmm_apply; the caller passes inputs and outputs.
 * It allocates no device memory (no hipMalloc, hipFree or other allocating
 * call): the per-apply workspace (tree arrays, grouped points and densities,
 * expansions, near-field partial sums, counters and error flags) is one fixed
 * array of LMFMM_NOALLOC_MAX_BYTES inside the library, one copy per GPU, held
 * until the process ends.  Its counters are cleared by a kernel at the start
 * of every call.
 *   - The plan's translation and near-field tables for the apply's geometry
 *     must exist: an earlier lmfmm_apply of the plan with the same geometry
 *     (same bounding box, or the same "domain" option, and the same levels)
 *     builds them.  Otherwise LMFMM_EINVAL and nothing is queued.
 *   - An apply whose workspace exceeds LMFMM_NOALLOC_MAX_BYTES returns
 *     LMFMM_EINVAL (the message states the size needed) before queuing anything.
 *   - The plan's device must be current.  Kernels are launched one by one (no
 *     graph); without the "domain" option the call waits for the bounding box
 *     as lmfmm_apply does.  The plan's statistics are not updated.
 *   - With "tree_sort" at "auto" the points are grouped by the counting sort,
 *     which needs the least workspace; "radix" is honoured.
 *   - Every call on one GPU shares that GPU's array: calls that overlap on a
 *     GPU (other streams, other host threads, other plans) race and give wrong
 *     results.  lmfmm_sync_status reports the error flag of the last such call
 *     only until the next one on that GPU. */
int lmfmm_apply_noalloc(lmfmm_plan plan, int64_t n_src, const double *src_xy, const void *q, int64_t n_tgt,
                        const double *tgt_xy, void *u, int nrhs, int precision, void *stream);

/* Transposed operator, no conjugation: v[r][j] = sum_i g_2^t(tgt_i, src_j) w[r][i].
 * Same arguments as lmfmm_apply with w: [nrhs][n_tgt] in, v: [nrhs][n_src] out. */
int lmfmm_apply_adjoint(lmfmm_plan plan, int64_t n_src, const double *src_xy, int64_t n_tgt,
                        const double *tgt_xy, const void *w, void *v, int nrhs, int precision,
                        void *stream);

/* Coordinate gradients of L = Re sum_r sum_i w[r][i] u[r][i], u = G q:
 *   dsrc: [2][n_src] float64 (dL/dx_j, dL/dy_j), dtgt: [2][n_tgt] float64.
 * The kernel's derivatives multiply the Sommerfeld integrand by i lam (x1),
 * s2 (y1), -i lam (x0), -s1 (y0).  Tree and expansions are recomputed. */
int lmfmm_grad_coords(lmfmm_plan plan, int64_t n_src, const double *src_xy, const void *q, int64_t n_tgt,
                      const double *tgt_xy, const void *w, double *dsrc, double *dtgt, int nrhs,
                      int precision, void *stream);

/* Brute-force direct sum on the GPU (every pair by contour quadrature, FP64
 * arithmetic, no tree); same arguments and result as lmfmm_apply. */
int lmfmm_direct(lmfmm_plan plan, int64_t n_src, const double *src_xy, const void *q, int64_t n_tgt,
                 const double *tgt_xy, void *u, int nrhs, int precision, void *stream);

/* Statistics of the last apply. */
typedef struct {
    int levels;            /* quadtree depth L                               */
    int order[32];         /* expansion order used at levels 0..L            */
    double root_x_lo;      /* root square [x_lo, x_lo+width] x [-w/2, w/2]    */
    double root_width;
    int64_t m2l_pairs;     /* box pairs translated by M2L (all levels)       */
    int64_t leaves_src;    /* leaf boxes covering the sources' bounding box   */
    int64_t leaves_tgt;
    int near_nodes_mid;    /* near-field quadrature nodes on the finite piece */
    int near_nodes_ray;    /* ... on each of the two rays                     */
    int m2l_classes;       /* translation classes with a table               */
    int64_t m2l_nodes;     /* quadrature nodes summed over all classes       */
    double table_seconds;  /* host wall time of the last M2L table rebuild   */
    /* Per kernel, indexed by LMFMM_K_*:
     *   kernel_flops: algorithmic real floating-point operations of the last
     *   apply (complex multiply-add = 8; translation and accumulation
     *   contractions counted over the box pairs and points the method
     *   defines, basis evaluations at 60 P per point; the near-field sweep
     *   at 32 per complex exponential plus 8 per right-hand side for every
     *   point of the interface leaves, node and sweep direction).  The leaf
     *   evaluation and sweep counts depend on the leaves' populations:
     *   lmfmm_get_stats reads them back and then synchronizes the device;
     * with the "timing" option, summed over the timed applies:
     *   kernel_ms: event-measured duration, kernel_launches: launches.     */
    double kernel_flops[8];
    double kernel_ms[8];
    int64_t kernel_launches[8];
    int64_t timed_applies;
    int64_t graph_applies;  /* applies run as a captured HIP graph (lifetime)  */
} lmfmm_stats;

/* Kernel indices of lmfmm_stats.kernel_*: bounding box and tree build (all
 * their kernels together), P2M, M2M, M2L (all levels in one launch),
 * near-field sweep, L2P + near field (or its gradient form), L2L; 7 is
 * unused. */
enum { LMFMM_K_TREE = 0, LMFMM_K_P2M = 1, LMFMM_K_M2M = 2, LMFMM_K_DOWN = 3, LMFMM_K_SWEEP = 4, LMFMM_K_L2P = 5,
       LMFMM_K_L2L = 6, LMFMM_K_OTHER = 7 };

int lmfmm_get_stats(lmfmm_plan plan, lmfmm_stats *stats);

/* Synchronize the stream and report a device-detected error of the plan's
 * last apply (points outside the fixed domain or their layer). */
int lmfmm_sync_status(lmfmm_plan plan, void *stream);

/* ---------------------------------------------------------------------------
 * Batched apply: many independent problems (own medium, points, densities).
 * Not in the paper: a throughput interface for uneven problem sizes.
 *
 * lmfmm_batch_create makes one plan per instance; order_set lists candidate
 * order floors (e.g. {12, 16, 20}) and tol the accuracy every candidate must
 * meet (the order rule of lmfmm_create enforces it).  On the first
 * lmfmm_batch_apply, and whenever the descriptors, nrhs or precision change,
 * the batch prepares:
 *   - each instance's bounding box is read once and pinned (later applies
 *     queue no host synchronisation);
 *   - each instance's (order floor, levels) comes from the tuning cache if it
 *     holds the instance's key (medium, size buckets, tol, nrhs, precision,
 *     order set), else an autotuner times every candidate with HIP events and
 *     keeps the fastest, then times the other near-field form (sweep or
 *     pairwise sum, plan option "near_sweep") at that choice; then the
 *     depth of the instances tuned now is capped at one and two levels below
 *     the deepest, the merged launch sequence is timed for each cap, and the
 *     fastest is kept (merged launches of one stage run together, so the
 *     deepest instance sets the number of per-level launches); the choices
 *     are added to the cache;
 *   - every instance's launch sequence is recorded and the launches of each
 *     stage (tree passes, P2M, M2M per level, M2L, L2L per level, near field,
 *     local evaluation) are merged into one launch over all instances, captured
 *     in a HIP graph.
 * Later calls with the same descriptors are one hipGraphLaunch on `stream`
 * with no host synchronisation.  Points rewritten in place must stay inside
 * the pinned bounding boxes: lmfmm_batch_sync_status reports any instance
 * whose points left it (its results are then invalid) and makes the next
 * apply prepare again.
 * inst: host array of n_inst descriptors with device pointers (read during
 * the call); all instances use the same nrhs and precision, and u must hold
 * [nrhs][n_tgt] elements of that precision.  Calls that overlap on one batch
 * are not allowed (a batch is not thread-safe).
 * Options (lmfmm_batch_set_option): "tune" 0/1 (default 1), "graph" 0/1
 * (default 1), "tune_cache" path of the tuning cache (one JSON object per
 * line; default: the environment variable LMFMM_TUNE_CACHE, else none),
 * "timing" 1/0/reset (launch the merged sequence with start/stop events per
 * launch and accumulate the durations per kernel class in
 * lmfmm_batch_stats); other keys are forwarded to every instance's plan
 * ("near_sweep" set this way also stops the tuner choosing the form).
 * --------------------------------------------------------------------------- */
typedef struct lmfmm_batch_s *lmfmm_batch;
typedef struct {
    int64_t n_src;
    const double *src_xy; /* device [2][n_src] */
    const void *q;        /* device [nrhs][n_src] */
    int64_t n_tgt;
    const double *tgt_xy; /* device [2][n_tgt] */
    void *u;              /* device [nrhs][n_tgt], overwritten */
} lmfmm_instance;

typedef struct {
    int launches;          /* merged kernel launches per apply               */
    int instances;
    int tuned_from_cache;  /* instances whose choice came from the cache     */
    double prepare_seconds;  /* host wall time of the last preparation      */
    /* by LMFMM_K_* class: algorithmic work of one apply summed over the
     * instances (as lmfmm_stats.kernel_flops); with "timing", the summed
     * event-measured durations and launches of the timed applies          */
    double kernel_flops[8];
    double kernel_ms[8];
    int64_t kernel_launches[8];
    int64_t timed_applies;
    int64_t graph_applies;
} lmfmm_batch_stats;

int lmfmm_batch_create(int n_inst, const double *k /* [n_inst][6] */, const double *d /* [n_inst] */,
                       const int *order_set, int n_orders, double tol, lmfmm_batch *out);
int lmfmm_batch_destroy(lmfmm_batch batch);
int lmfmm_batch_set_option(lmfmm_batch batch, const char *key, const char *value);
int lmfmm_batch_apply(lmfmm_batch batch, const lmfmm_instance *inst, int nrhs, int precision, void *stream);
/* The autotuner's choice for instance i: order floor, levels, near-field form
 * (1: the x-ordered sweep, 0: the pairwise sum) and its measured time per
 * apply (us).  Null out-pointers are skipped. */
int lmfmm_batch_get_choice(lmfmm_batch batch, int i, int *order, int *levels, double *us, int *near_sweep);
int lmfmm_batch_get_stats(lmfmm_batch batch, lmfmm_batch_stats *stats);
/* Synchronize the stream; LMFMM_EDOMAIN if any instance's points left the
 * bounding box the batch was prepared for or their layer (the next apply then
 * prepares again), else LMFMM_OK. */
int lmfmm_batch_sync_status(lmfmm_batch batch, void *stream);

const char *lmfmm_status_string(int status);
const char *lmfmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LMFMM_H */
