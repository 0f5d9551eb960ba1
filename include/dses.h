/*
 * dses.h -- C ABI of the MI355X (gfx950) implementation of Direct Semi-Exhaustive
 * Search (DSES) for partial-to-full rigid point-cloud registration
 * (Cheng, Papozov, Helmick, Tjersland, arXiv 2502.00115).
 *
 * The library runs the data-parallel hot path of the method on one GPU: for every
 * rotation R of a caller-given candidate list it
 *   1. votes every rotated point-pair translation y_j - R x_i into a translation
 *      lattice of pitch delta and takes the mode t* and its frequency M
 *      (Lemma 2, Eq. (5); first loop of Alg. 2);
 *   2. scores the candidate {R, t*} directly: d_i = min_j ||R x_i + t* - y_j||,
 *      inliers = #{d_i < eps}, error = sum_i rho(d_i) for the chosen robust metric
 *      (Eq. (1)/(2); error loop of Alg. 2 with q = 0, i.e. every candidate scored);
 *   3. returns the candidate with the smallest error (return step of Alg. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Point clouds are row-major float32 xyz arrays: src is N x 3 (the partial
 *    observation X), tgt is M x 3 (the full reference Y).
 *  - Rotations are row-major float32 3x3 matrices, K x 9, mapping the source frame
 *    into the reference frame: a candidate transforms x as R x + t.
 *  - Pointers are host pointers unless DSES_DEVICE_PTRS is set in the options flags,
 *    in which case src/tgt/rotations (and dses_options.records) are device pointers
 *    on the library's device (e.g. torch tensors' data_ptr()).
 *  - The caller owns every buffer it passes; the library only reads inputs during
 *    the call (for dses_server_submit: until dses_server_wait returns for that
 *    request) and never frees caller memory.
 *  - Every call returns a dses_status; on failure a message is available from
 *    dses_last_error() (thread-local) and `out` is left untouched.
 *
 * Translation lattice and ROUND (Alg. 2: the rounded pair translation y_j - R x_i)
 * ----------------------------------------------------------------------------
 * The vote array spans the translation box [t_min, t_max] (default [-1, 1]^3;
 * the paper bounds it by the search range of its experiments, Sec. V).  Its bins
 * are the lattice points b*delta with, per axis a,
 *     k_lo_a = ceil(t_min_a/delta - 1e-4),  k_hi_a = floor(t_max_a/delta + 1e-4)
 * (double precision), size_a = k_hi_a - k_lo_a + 1.  A pair votes for the nearest
 * lattice point, halves rounded up: b_a = floor((y_a - p_a)/delta + 1/2) with
 * p = R x (Lemma 2, Eq. (5)), and only if b lies in the box.  The kernels take
 * this decision on integers (the paper fixes no precision).  With
 * S_F = (1/delta) 2^F in double, F = 16 on x and y, and on z F = 15 when the
 * counters are 16-bit (the library proves no bin can reach 2^16 votes) or 16:
 *     Y_a = rint(y_a S_F + (1/2 - k_lo_a) 2^F)            (reference, once)
 *     p_a = (R[a][0] x_x + R[a][1] x_y) + R[a][2] x_z     (double, per rotation)
 *     P_a = rint(p_a S_F), saturated at +-2^30 (no such source value can vote)
 *     c_a = floor((Y_a - P_a) / 2^F)                      (box-relative bin)
 * every product and sum one rounded double operation, rint rounding halves to
 * even, the difference exact int32 arithmetic; a pair votes iff
 * 0 <= c_a < size_a on every axis.  Each rounding moves u + 1/2 by at most half
 * a unit, so a pair whose exact u + 1/2 lies within 2^-F bins (at most 3.1e-5) of an
 * integer may be counted in the neighbouring bin.  The integers stay apart in 32
 * bits because every reference coordinate is limited to |y| <= (2^13 - K - 8)
 * delta (K the largest |k_lo_a| or |k_lo_a + size_a|; at most 1e4) and every
 * source coordinate to |x| <= 1e4: larger ones are rejected with DSES_E_INVAL.
 * The mode is the bin with the
 * largest count; ties go to the lowest linear index
 * ((c_x * size_y + c_y) * size_z + c_z).  The returned translation is
 * t_a = (float)(c_a + k_lo_a) * delta (no refinement: the paper's answer is exact
 * only up to the discretisation delta).
 *
 * Metrics (Eq. (1) leaves the norm free; Sec. IV-B uses a truncated norm)
 * ------------------------------------------------------------------------
 *   DSES_TRUNC_L2  error = sum_i min(d_i, tau), d_i the Euclidean NN distance
 *   DSES_INLIERS   error = N - inliers  (the L0^{m1} objective of Eq. (3), Thm. 3)
 *   DSES_TLS       error = sum_i min(d_i^2, tau^2)
 *   DSES_TRUNC_L1  error = sum_i min(min_j ||q_i - y_j||_1, tau)
 *   DSES_TRUNC_LP  error = sum_i min(d_i, tau)^p, p in (0, 1] (dses_options.p; the
 *                  Lp, p < 1, sparsity objectives that Sec. III admits)
 *   DSES_VOTES     no scoring: candidates are ranked by their mode count M_k alone
 *                  (Thm. 3: under its separation condition M_k is the L0^{m1}
 *                  inlier count of {R_k, t_k}); records and results carry
 *                  error 0 and inliers = M_k, so the selection is the largest
 *                  M_k, ties to the lower rotation index
 * inliers always counts d_i < eps with the Euclidean d_i.  All scoring runs in
 * float32; ties in the final selection go to more inliers, then the lower
 * rotation index (the paper is silent on ties).
 */
#ifndef DSES_H
#define DSES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DSES_OK = 0,
    DSES_E_INVAL = -1,        /* bad argument: NULL pointer, n/m/k <= 0, eps <= 0 or
                                 non-finite, non-finite coordinate, coordinate too large
                                 for the lattice, non-orthonormal rotation
                                 (|R^T R - I|_max > 1e-4), empty box, bad option      */
    DSES_E_NOCANDIDATE = -2,  /* no rotation received a vote inside the box            */
    DSES_E_NOMEM = -3,        /* device allocation failed / request exceeds a budget   */
    DSES_E_TIMEOUT = -4,      /* dses_server_wait timed out                            */
    DSES_E_DEVICE = -5,       /* HIP runtime error, or no usable gfx950 device          */
    DSES_E_STATE = -6         /* wrong handle state (e.g. unknown or consumed request)  */
} dses_status;

typedef enum {
    DSES_TRUNC_L2 = 0,
    DSES_INLIERS = 1,
    DSES_TLS = 2,
    DSES_TRUNC_L1 = 3,
    DSES_TRUNC_LP = 4,        /* dses_register / dses_register_resident only          */
    DSES_VOTES = 5            /* dses_register / dses_register_resident only          */
} dses_metric;

/* How the per-candidate nearest-neighbour term of Eq. (2) is evaluated. */
typedef enum {
    DSES_SCORER_AUTO = 0,   /* GRID, or DF when the target handle carries a field    */
    DSES_SCORER_BRUTE = 1,  /* every reference point per source point (the error
                               loop of Alg. 2 as printed, a brute-force search)       */
    DSES_SCORER_GRID = 2,   /* exact: only reference points within r = max(eps, tau)
                               can change rho or the inlier test, found through a
                               uniform cell grid of pitch >= r; same result as BRUTE  */
    DSES_SCORER_DF = 3      /* voxel distance field of the reference (approximate,
                               see dses_target_create); TRUNC_L1 is not supported     */
} dses_scorer;

/* How a distance-field scorer reads the field at a query q (dses_target_create). */
typedef enum {
    DSES_DF_NEAREST = 0,    /* the value of the voxel containing q                    */
    DSES_DF_TRILINEAR = 1   /* linear interpolation between the 8 voxel centres around
                               q along each axis (r at centres outside the grid)       */
} dses_df_lookup;

#define DSES_DEVICE_PTRS 0x1u   /* inputs (and records) are device pointers            */
#define DSES_TIMING 0x2u        /* time each kernel with HIP events (dses_kernel_stats) */
#define DSES_BATCH_TUNE 0x4u    /* dses_register_batch: autotune the launch layout (below) */

typedef struct {
    uint32_t struct_size;     /* sizeof(dses_options); 0-filled fields mean defaults  */
    uint32_t flags;           /* DSES_DEVICE_PTRS | DSES_TIMING                         */
    float delta_t;            /* translation bin pitch; 0 -> eps                        */
    float tau;                /* truncation of the robust metrics; 0 -> eps             */
    float t_min[3];           /* translation box; t_min == t_max == 0 -> [-1, 1]^3      */
    float t_max[3];
    int32_t scorer;           /* dses_scorer; 0 -> AUTO                                 */
    int32_t top_k;            /* 0..DSES_TOPK_MAX best candidates to return in topk      */
    void *stream;             /* hipStream_t to run on; NULL -> the library's stream    */
    void *records;            /* optional: K dses_record, one per rotation, filled on
                                 DSES_OK (host memory, or device with DSES_DEVICE_PTRS) */
    void *topk;               /* optional: top_k dses_candidate, best first in the
                                 selection order (error, then more inliers, then lower
                                 rotation index; the first equals the result); entries
                                 past the number of valid rotations have rot_index -1.
                                 Host memory, or device with DSES_DEVICE_PTRS          */
    float q;                  /* pruning of Alg. 2 (Sec. IV-B): 0 -> score every
                                 candidate; q in (0, 1] -> vote all rotations, then
                                 score only those whose mode count M_k >= q M* (M* =
                                 the largest M_k; compared in double precision), the
                                 others keep their bin and votes with error +inf and
                                 0 inliers and are never selected (not with
                                 DSES_VOTES)                                          */
    float p;                  /* exponent of DSES_TRUNC_LP, in (0, 1]; 0 -> 0.5        */
    int32_t lane_group;       /* vote layout (sources up to 16,384 points): reference
                                 points per lane group, 16, 32 or 64 (a wave holds
                                 64 / lane_group copies of the group, each streaming
                                 alternate 4-source pieces of its window); 0 ->
                                 chosen per call from the sizes and the reference's
                                 extent.  Results do not depend on it; other values
                                 are DSES_E_INVAL                                     */
    int32_t df_lookup;        /* dses_df_lookup of the DF scorer; 0 -> NEAREST         */
} dses_options;

#define DSES_TOPK_MAX 64

/* One scored candidate {R_k, t_k} (28 bytes), for the top-k output. */
typedef struct {
    int32_t rot_index;        /* index into the rotation list, -1: none               */
    int32_t inliers;
    float error;
    uint32_t votes;           /* M of t_k                                             */
    float t[3];               /* t_k = b* delta                                       */
} dses_candidate;

/* Result of one registration. */
typedef struct {
    float R[9];               /* selected rotation (copied from the list)             */
    float t[3];               /* its mode translation t* (a lattice point)            */
    int32_t rot_index;        /* index into the rotation list                         */
    int32_t inliers;          /* #{d_i < eps}                                         */
    float error;              /* e(R, t*) under the metric                            */
    uint32_t votes;           /* M: vote count of t*                                  */
    int32_t n_valid;          /* rotations that received at least one in-box vote     */
} dses_result;

/* Per-rotation candidate record (24 bytes), optional output. */
typedef struct {
    int32_t bin[3];           /* mode bin b* (t* = b* delta); undefined if votes == 0 */
    uint32_t votes;           /* M; 0 marks a rotation with no in-box vote (invalid)  */
    int32_t inliers;
    float error;              /* +inf for invalid rotations                           */
} dses_record;

/* Cumulative HIP-event kernel timings (DSES_TIMING), per kernel family. */
typedef struct {
    double vote_score_ms;     /* fused vote + mode + score kernel(s)                   */
    double score_ms;          /* separate scoring kernel(s), if any                    */
    double select_ms;         /* candidate selection                                   */
    double stage_ms;          /* input staging / grids / distance fields               */
    int64_t vote_score_launches;
    int64_t score_launches;
    int64_t pairs_voted;      /* sum of N*M over rotations swept (algorithmic)        */
    int64_t pairs_scored;     /* sum of N*M over candidates scored by BRUTE            */
    int64_t candidates;       /* rotations swept                                      */
} dses_kstats;

/* ---------------------------------------------------------------------------- */
/* Library                                                                       */
/* ---------------------------------------------------------------------------- */

/* Thread-local description of the last failure in this thread ("" if none). */
const char *dses_last_error(void);

/* Select and initialise the HIP device (default 0).  Optional: every entry point
 * initialises device 0 on first use.  Returns DSES_E_DEVICE without a gfx950 GPU. */
dses_status dses_init(int32_t device);

/* Library version string. */
const char *dses_version(void);

/* Read (and with reset != 0 clear) the DSES_TIMING kernel statistics. */
dses_status dses_kernel_stats(dses_kstats *out, int32_t reset);

/* Fault injection, for tests of the error paths: of the library's next device
 * and pinned-host allocations (every one it makes, in any thread), the first
 * `skip` succeed and the `count` after them fail as if out of memory (the entry
 * point that made the allocation reports DSES_E_NOMEM or DSES_E_DEVICE and
 * leaves every object it was given usable).  (0, 0) turns injection off.
 * Negative arguments: DSES_E_INVAL.  Process-wide; not for production use. */
dses_status dses_debug_fail_allocs(int32_t skip, int32_t count);

/* ---------------------------------------------------------------------------- */
/* Plain registration (Alg. 2 with q = 0)                                        */
/* ---------------------------------------------------------------------------- */

/* Register src (n x 3) to tgt (m x 3) over the k rotations; synchronous on the
 * chosen stream.  Requires n*m < 2^31.  opt may be NULL (all defaults, host
 * pointers).  Writes *out and, if opt->records != NULL, k records. */
dses_status dses_register(const float *src, int64_t n, const float *tgt, int64_t m,
                          const float *rotations, int64_t k, float eps, dses_metric metric,
                          const dses_options *opt, dses_result *out);

/* dses_register for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and records as dses_register, with these limits:
 *  - src, tgt, rotations (and opt->records, if given) are device pointers:
 *    opt->flags must be exactly DSES_DEVICE_PTRS; top_k and q must be 0; the DF
 *    scorer is not available (it needs a resident target);
 *  - every device buffer of the call (staged reference, cell grid, source-sort
 *    slots, records unless opt->records is given, result, status) comes from one
 *    static device array of dses_noalloc_scratch_bytes() (64 MiB) per GPU; the
 *    call makes no hipMalloc, hipFree or pinned-host allocation.  A call that
 *    needs more returns DSES_E_NOMEM with a message naming the limit (the
 *    scene-scale registration, 4,096 x 16,384 points and 294,912 rotations,
 *    needs about 33 MiB);
 *  - the array is shared by every call on that GPU and keeps the last call's
 *    contents; calls are serialised by the library and synchronous, but work of
 *    another process or library writing the same addresses would race.
 * Host working memory for the reference's sort and cell grid is ordinary heap. */
dses_status dses_register_noalloc(const float *src, int64_t n, const float *tgt, int64_t m,
                                  const float *rotations, int64_t k, float eps,
                                  dses_metric metric, const dses_options *opt, dses_result *out);

/* Size in bytes of the per-GPU scratch array of dses_register_noalloc. */
size_t dses_noalloc_scratch_bytes(void);

/* Alg. 1, the pure exhaustive search, as a baseline: every rotation of the list
 * with every lattice translation b delta_t of the box, each scored like a DSES
 * candidate (BRUTE or GRID scorer; any metric but DSES_VOTES).  opt->records gets
 * per rotation its best translation (smaller error, more inliers, lower linear
 * index of b, x slowest) with votes = 1; *out the best pose overall (ties to the
 * lower rotation index).  Cost: k x (box bins) x n nearest-neighbour queries.
 * Requires n <= 12288 and at most 2^31 - 1 bins; top_k and q must be 0. */
dses_status dses_register_exhaustive(const float *src, int64_t n, const float *tgt, int64_t m,
                                     const float *rotations, int64_t k, float eps,
                                     dses_metric metric, const dses_options *opt,
                                     dses_result *out);

/* ---------------------------------------------------------------------------- */
/* Resident data: reference clouds (with optional distance field) and rotation   */
/* lists kept in device memory across calls (the serving workload keeps them).   */
/* ---------------------------------------------------------------------------- */
typedef struct dses_target dses_target;
typedef struct dses_rotset dses_rotset;

typedef struct {
    uint32_t struct_size;
    uint32_t flags;           /* DSES_DEVICE_PTRS: tgt is a device pointer            */
    float df_trunc;           /* > 0: build a distance field truncated at this radius  */
    int32_t df_res;           /* field resolution per axis (0 -> 128)                  */
} dses_target_opts;

/* Upload a reference cloud (m x 3).  With df_trunc = r > 0 also build its voxel
 * distance field: a df_res^3 float32 grid over the reference AABB padded by r,
 * voxel centres c = lo + (idx + 1/2) h, value min(min_j ||c - y_j||, r), where in
 * float32  lo_a = min_j y_a - r,  h_a = ((max_j y_a + r) - lo_a) / df_res.
 * A DF query q (formed in float32 as R x + t) reads, with DSES_DF_NEAREST, the
 * voxel idx_a = floor((q_a - lo_a)/h_a) (evaluated as floorf((q_a - lo_a) *
 * (1.0f / h_a))); outside the grid its value is r.  With DSES_DF_TRILINEAR it
 * interpolates linearly along each axis between the values at the 8 voxel
 * centres around q, u_a = (q_a - lo_a)/h_a - 1/2, a centre outside the grid
 * counting as r (outside the padded box every point is farther than r from the
 * reference); the interpolant is continuous in q.  DF scoring requires
 * r == max(eps, tau) of the registration. */
dses_status dses_target_create(const float *tgt, int64_t m, const dses_target_opts *opt,
                               dses_target **out);
dses_status dses_target_destroy(dses_target *t);
/* Copy the distance field (df_res^3 floats, x slowest) and its lo[3]/h[3] to host
 * buffers; for checking.  Returns DSES_E_STATE if the target has no field. */
dses_status dses_target_field(const dses_target *t, float *field, float *lo, float *h);

/* Alg. 2's rotation grid: (2K+1)^3 rotations R = C Rz(theta) Ry(phi) Rx(xi) for
 * theta, phi, xi in {-K step, ..., +K step} (radians), theta slowest and xi
 * fastest (the loop order of Alg. 2); C = center (row-major 3x3, NULL: identity),
 * the initial guess of a local registration.  The Euler convention (intrinsic
 * z-y-x) is this library's reading; the paper does not fix one.  Host only: out
 * holds (2K+1)^3 x 9 floats; needs no device.  0 <= K <= 200, step > 0. */
dses_status dses_rotations_euler(const float *center, int32_t K, float step, float *out);

/* Upload a rotation list (k x 9) once. */
dses_status dses_rotations_create(const float *rotations, int64_t k, uint32_t flags,
                                  dses_rotset **out);
dses_status dses_rotations_destroy(dses_rotset *r);

/* dses_register against resident data (tgt/rotations arguments replaced). */
dses_status dses_register_resident(const dses_target *tgt, const dses_rotset *rots,
                                   const float *src, int64_t n, float eps, dses_metric metric,
                                   const dses_options *opt, dses_result *out);

/* ---------------------------------------------------------------------------- */
/* Batched registration: many independent registrations in one persistent       */
/* launch (captured once in a HIP graph and replayed).                           */
/* ---------------------------------------------------------------------------- */
typedef struct {
    const float *src;         /* n x 3 */
    int64_t n;
    const float *tgt;         /* m x 3 (ignored when target != NULL) */
    int64_t m;
    const float *rotations;   /* k x 9 (ignored when rotset != NULL) */
    int64_t k;
    const dses_target *target;   /* optional resident reference */
    const dses_rotset *rotset;   /* optional resident rotations */
    float eps;
    int32_t metric;
    float delta_t, tau;       /* 0 -> eps */
    float t_min[3], t_max[3]; /* both 0 -> [-1, 1]^3 */
    void *records;            /* optional k dses_record */
} dses_problem;

typedef struct {
    uint32_t struct_size;
    uint32_t flags;           /* DSES_DEVICE_PTRS | DSES_TIMING | DSES_BATCH_TUNE */
    int32_t scorer;           /* dses_scorer for every problem */
    int32_t use_graph;        /* 1: capture the launch in a HIP graph and replay it */
    int32_t tile_rot;         /* rotations per work item; 0 -> tuned or default layout */
    int32_t vote_parts;       /* vote work units per lane group (parts of its
                                 stream window, 1..16); 0 -> tuned or automatic
                                 (64 / groups, 1..8, per problem)                   */
    void *stream;
    int32_t df_lookup;        /* dses_df_lookup for DF-scored problems; 0 -> NEAREST  */
} dses_batch_opts;

/* Register every problem; results (and records) are identical to running each
 * problem alone with dses_register, whatever the launch layout.  Synchronous.
 *
 * Launch layout.  The persistent launch takes (instance, rotation tile) items from
 * one work list, most expensive first.  Two knobs shape it: the work-list
 * granularity (tiles sized so that the list holds about `items_per_cu` items per
 * compute unit, unless tile_rot fixes the tile) and vote_parts (into how many work
 * units the vote splits each lane group's stream window: 16, 32 or 64 reference
 * points, chosen per problem as with dses_options.lane_group = 0, against the
 * window of x-sorted sources; the waves of a workgroup take units dynamically).
 * With DSES_BATCH_TUNE the call first times the sweep kernel alone on this batch
 * for candidate layouts (items_per_cu in {6, 12, 24, 48, 96}, then vote_parts in
 * {1, 2, 4, 8}, one coordinate at a time), keeps the fastest for every later batch
 * of the same class (same count and scorer, same power-of-two bucket of total
 * pairs, of mean source size and of mean rotation count), and then runs the batch
 * with it.  Without the flag a batch uses its class's tuned layout if one exists,
 * else the default (items_per_cu 24, vote_parts automatic). */
dses_status dses_register_batch(const dses_problem *probs, int32_t count,
                                const dses_batch_opts *opt, dses_result *out,
                                dses_status *status);

typedef struct {
    int32_t items_per_cu;     /* work-list granularity used (0 when tile_rot fixed it) */
    int32_t vote_parts;       /* vote work units per lane group used (0: automatic)    */
    int32_t n_items;          /* work items in the launch                             */
    int32_t source;           /* 0 default, 1 tuned by this call, 2 tuned earlier for
                                 this class, 3 given by the caller                    */
    int32_t candidates;       /* layouts timed by this call (source 1)                */
    float sweep_ms;           /* sweep kernel time of the chosen layout when tuned    */
} dses_batch_config;

/* Launch layout of this thread's last successful dses_register_batch call. */
dses_status dses_batch_last_config(dses_batch_config *out);

/* ---------------------------------------------------------------------------- */
/* Diagnostics                                                                  */
/* ---------------------------------------------------------------------------- */
/* LDS atomic throughput of this device, the ceiling of the vote's counter
 * increments (vendors do not publish it): one 1,024-thread workgroup per CU with
 * a 160 KB LDS allocation, every lane issuing ds_add_u32 of 1; pattern 0 sends
 * each wave's 64 lanes to 64 distinct banks, pattern 1 to pseudo-random words
 * of the allocation (the vote's pattern).  Returns increments per second for the
 * whole device and, if per_cu_per_cycle is not NULL, per CU per clock cycle (at
 * the device's reported peak clock).  Takes tens of milliseconds. */
dses_status dses_measure_lds_atomics(int32_t pattern, double *adds_per_second,
                                     double *per_cu_per_cycle);

/* ---------------------------------------------------------------------------- */
/* Serving: a request loop with memory-based admission and continuous batching. */
/* ---------------------------------------------------------------------------- */
typedef struct dses_server dses_server;

typedef struct {
    uint32_t struct_size;
    uint32_t flags;
    int64_t memory_budget;    /* bytes of per-request device memory in flight (0: 1 GiB) */
    int32_t max_inflight;     /* requests on the device at once (0: 64)               */
    int32_t scorer;           /* dses_scorer for every request                         */
    float aging;              /* scheduling: a request's priority is its estimated
                                 remaining GPU time minus aging x its age (smallest
                                 first); 0 -> 3.0 (on the serving workload: median
                                 and mean latency below one launch per request in
                                 arrival order, p99 within 1%), < 0 -> 0 (shortest
                                 remaining work first), very large -> first come
                                 first served                                      */
    int32_t slice_mpairs;     /* work per slice (one batched launch), in millions of
                                 rotated point pairs; 0 -> 48000                       */
} dses_server_opts;

dses_status dses_server_create(const dses_server_opts *opt, dses_server **out);
/* Queue a registration of host src (n x 3, n <= 16,384) against resident data;
 * the source is copied at submit time.  Returns a request id.
 * opt (NULL: defaults) sets this request's delta_t, tau, translation box,
 * scorer (0: the server's), df_lookup, and optionally asks for its records
 * (opt->records: k dses_record) and its top_k best candidates (opt->topk);
 * both are host buffers the caller keeps valid until dses_server_wait returns
 * for the request, filled before the request is reported finished.  flags
 * (other than 0), stream, q, p and lane_group are plain-path options and must be
 * 0; DSES_TRUNC_LP and DSES_VOTES are plain-path metrics.  The result equals that
 * of dses_register_resident with the same options, whatever else is served. */
dses_status dses_server_submit(dses_server *srv, const dses_target *tgt,
                               const dses_rotset *rots, const float *src, int64_t n, float eps,
                               dses_metric metric, const dses_options *opt, uint64_t *req_id);
/* Wait up to timeout_ms (< 0: forever) for a request.  On DSES_OK the request is
 * consumed: *out (if *req_status is DSES_OK), *req_status, and if not NULL its
 * time from submission to admission to the device (*queue_s) and to completion
 * (*total_s), in seconds, are written, and the id is forgotten (a later wait,
 * poll, timing or cancel of it returns DSES_E_STATE). */
dses_status dses_server_wait(dses_server *srv, uint64_t req_id, int32_t timeout_ms,
                             dses_result *out, dses_status *req_status, double *queue_s,
                             double *total_s);
/* Non-blocking: 1 if finished, 0 if pending, < 0 on error (DSES_E_STATE for an
 * unknown or consumed id). */
int32_t dses_server_poll(dses_server *srv, uint64_t req_id);
/* Queue and total latency (seconds) of a finished request not yet consumed by
 * dses_server_wait. */
dses_status dses_server_timing(dses_server *srv, uint64_t req_id, double *queue_s,
                               double *total_s);
/* Withdraw a request that is still queued (not yet admitted to the device): it is
 * consumed and never runs.  DSES_E_STATE if it is unknown, consumed, already on
 * the device or finished (wait for it instead). */
dses_status dses_server_cancel(dses_server *srv, uint64_t req_id);
dses_status dses_server_destroy(dses_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* DSES_H */
