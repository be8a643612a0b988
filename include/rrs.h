/*
 * rrs.h -- C ABI of librrs: Refined Random Search (RRS) projection-based
 * depths on AMD Instinct MI355X (gfx950).
 *
 * Method: Leone, Mozharovskyi, Bounie, "Massive parallelization of
 * projection-based depths" (arXiv 2506.08262).  For every query z_q (a row of
 * Z) the library approximates
 *
 *     D(z_q | X) = inf over unit u of D(z_q.u | X u)          (Definition 2)
 *
 * by RRS (Alg. 1; parallel form Alg. 4 / Alg. S5): r = n_refine refinements
 * of m_dir = ceil(K / r) random directions each -- uniform on the sphere in
 * the first refinement (Alg. S1), then uniform in angle inside a spherical cap
 * of half-angle (pi/2) * cap_shrink^(l-1) around the query's current best
 * direction (Alg. S4) -- keeping the smallest univariate depth found
 * (Corollary 1: every value returned is an upper bound of the exact depth).
 * The univariate depths are those of Sec. 2 (halfspace, projection,
 * asymmetric projection).  Directions come from a counter-based Philox4x64-10
 * stream keyed by (seed, query index), so a query's result does not depend on
 * which other queries share the call.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  X      : n x d data, row-major binary64 (row i = point x_i).
 *  Z      : m x d queries, row-major binary64.  (m is the number of queries;
 *           the number of directions per refinement is ceil(K / n_refine).)
 *  K      : total directions per query, >= 1; r * ceil(K/r) are evaluated.
 *  n_refine: number of refinements r, >= 1.
 *  cap_shrink: alpha in (0, 1], the cap half-angle factor per refinement.
 *  seed   : Philox key word 0.
 *  depth  : m outputs, binary64, written only when the call returns RRS_OK.
 *  opts   : may be NULL (host pointers, default stream, no optional outputs).
 *
 * Memory: with opts->device_ptrs == 0 every array is host memory and the call
 * returns after the result is in place.  With device_ptrs != 0 every array
 * (X, Z, outputs, optional outputs) is device memory on the current HIP
 * device; work is issued on opts->stream and the call still synchronises that
 * stream before returning.  The caller owns all arrays; the library keeps no
 * pointer after return.  The library owns a per-device workspace that grows
 * on demand and is released by rrs_release_workspace().
 *
 * Errors: every entry point returns a status and never aborts; the text of
 * the last failure on the calling thread is available from rrs_last_error().
 * RRS_E_INVAL: a NULL pointer with a positive size, n < 1, d < 2, K < 1,
 * n_refine < 1, cap_shrink outside (0, 1], a non-finite value in X or Z (host
 * pointers only), or an unknown precision.  m == 0 is a no-op returning RRS_OK.
 * RRS_E_NOMEM: device memory could not be obtained.  RRS_E_DEVICE: a HIP
 * error (text in rrs_last_error).  Calls from several threads are serialised.
 */
#ifndef RRS_H
#define RRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RRS_OK = 0,
    RRS_E_INVAL = 1,
    RRS_E_NOMEM = 2,
    RRS_E_DEVICE = 3,
    RRS_E_BUSY = 4,       /* rrs_wait timed out */
    RRS_E_CANCELLED = 5,  /* the request's context was destroyed before it ran */
    RRS_E_INTERNAL = 6
} rrs_status;

/* Arithmetic of the projection step (every notion).
 * RRS_F64: every projection is the binary64 fused multiply-add chain over
 *   coordinates 0..d-1 of the shared recipe, so counts, order statistics and
 *   depths are exact (bit-identical to the FP64 oracle).
 * RRS_F32_RECHECK: projections of the mean-centred data on the matrix cores
 *   in binary32 (v_mfma_f32_32x32x2_f32).  Halfspace depth takes a sign from
 *   that value only when it exceeds a rigorous error margin and recomputes
 *   the pair with the binary64 recipe otherwise; projection and asymmetric
 *   projection depth locate each order statistic (median, MAD, MAD_+) on the
 *   binary32 values and recompute only the values inside a rigorous window
 *   around it in binary64.  Counts, depths and the RRS trajectory are
 *   identical to RRS_F64.
 * RRS_BF16_RECHECK: as RRS_F32_RECHECK, with the products from two-term
 *   bfloat16 splits of the centred data and of the directions (three bf16
 *   products per K step on v_mfma_f32_32x32x16_bf16, binary32 accumulation).
 *   Identical to RRS_F64.  For halfspace depth, refinements l >= 2 also cull
 *   the points whose sign is the same for every direction of the cap (decided
 *   from the pole's projection and a rigorous bound), which changes no count.
 * RRS_F32_PLAIN: the binary32 matrix-core projections decide everything by
 *   themselves (signs, with a zero counting on both sides; order statistics),
 *   without recheck; results may differ from RRS_F64 where values are within
 *   the binary32 rounding error, and the trajectory may then differ too.
 * The matrix-core forms need ceil(K / n_refine) < 65536 and m <= 65535. */
typedef enum {
    RRS_F64 = 0,
    RRS_F32_RECHECK = 1,
    RRS_BF16_RECHECK = 2,
    RRS_F32_PLAIN = 3
} rrs_precision;

typedef struct {
    int32_t precision;        /* rrs_precision; default RRS_F64 */
    int32_t device_ptrs;      /* 0: host arrays; 1: device arrays */
    void *stream;             /* hipStream_t for device_ptrs == 1 (NULL: default) */
    int64_t query_offset;     /* stream index of Z's first row (default 0) */
    double *poles;            /* optional out [m x d]: final pole per query */
    int64_t *trace;           /* optional out [m x n_refine x 3]: per refinement
                                 j*, improved (0/1), minimum (int64 count for
                                 halfspace, binary64 bits otherwise) */
    size_t workspace_limit;   /* bytes the per-refinement scratch may use;
                                 0: library default */
    uint32_t flags;           /* RRS_FLAG_* (default 0) */
    uint32_t reserved;        /* must be 0 */
} rrs_opts;

/* flags: RRS_FLAG_GRAPH -- the call's device work (data preparation and the
 * whole refinement chain) is captured once into a HIP graph and replayed by
 * later calls with the same arguments (sizes, hyper-parameters, seed,
 * precision, pointers and stream); needs device_ptrs == 1 and no profiling.
 * Replays run exactly the captured kernels, so results are identical to the
 * eager calls.  rrs_release_workspace() drops the cached graphs. */
#define RRS_FLAG_GRAPH 1u

/* flags: RRS_FLAG_FIRST_CAP -- the first refinement draws its directions like
 * the later ones (Alg. S4, angle-uniform in the cap of half-angle pi/2 around
 * the initial direction e1), the literal reading of the algorithms' first
 * cap, instead of uniformly on the whole sphere (Alg. S1, the default; the
 * main text's description of the first step).  The two agree in law on the
 * hemisphere only up to the angle-uniform versus area-uniform weighting, and
 * the hemisphere misses half of the directions D_AP needs (D_AP is not
 * symmetric under u -> -u).  Provided to study that reading. */
#define RRS_FLAG_FIRST_CAP 2u

/* flags: RRS_FLAG_AREA_CAP -- the cap directions of refinements l >= 2 (and
 * of refinement 1 with RRS_FLAG_FIRST_CAP) are uniform in area on the cap
 * (the polar angle has density proportional to sin^(d-2)) instead of
 * Alg. S4's angle-uniform law; the polar angle comes from Newton's method on
 * the cap's area function, computed by a series that converges only below
 * the hemisphere: RRS_E_INVAL unless cap_shrink <= 0.99 and
 * RRS_FLAG_FIRST_CAP is off.  Both laws give every direction of the cap
 * positive density; the paper's text describes the cap as sampled
 * uniformly. */
#define RRS_FLAG_AREA_CAP 4u

/* Halfspace (Tukey) depth, Sec. 2: min(#{x_i.u <= z.u}, #{x_i.u >= z.u}) / n,
 * minimised over the RRS directions.  count (may be NULL) receives the
 * integer minimum count per query; depth = count / n. */
rrs_status rrs_depth_halfspace(const double *X, int64_t n, int64_t d,
                               const double *Z, int64_t m, int64_t K,
                               int32_t n_refine, double cap_shrink, uint64_t seed,
                               double *depth, int64_t *count, const rrs_opts *opts);

/* Projection depth, Sec. 2: (1 + |z.u - med(Xu)| / MAD(Xu))^-1 minimised over
 * the RRS directions; MAD = med |x_i.u - med(Xu)|.  MAD == 0 gives 1 when
 * z.u == med(Xu), else 0. */
rrs_status rrs_depth_projection(const double *X, int64_t n, int64_t d,
                                const double *Z, int64_t m, int64_t K,
                                int32_t n_refine, double cap_shrink, uint64_t seed,
                                double *depth, const rrs_opts *opts);

/* Asymmetric projection depth, Sec. 2: (1 + (z.u - med(Xu))_+ / MAD_+(Xu))^-1
 * minimised over the RRS directions; MAD_+ is the median of the strictly
 * positive deviations x_i.u - med(Xu).  No positive deviation gives 1 when
 * z.u <= med(Xu), else 0. */
rrs_status rrs_depth_apd(const double *X, int64_t n, int64_t d,
                         const double *Z, int64_t m, int64_t K,
                         int32_t n_refine, double cap_shrink, uint64_t seed,
                         double *depth, const rrs_opts *opts);

/* Mahalanobis depth with the moment estimates, D_M(L) (Sec. "Center-outward
 * ordering precision and depth benchmark": the closed-form comparator of the
 * ranking study): (1 + (z - mu)' Sigma^-1 (z - mu))^-1 with mu the mean of X
 * and Sigma its maximum-likelihood covariance (divisor n), all in binary64 on
 * the device (covariance and quadratic forms on the FP64 matrix cores).  Not
 * an RRS depth: no directions.  Memory conventions as the calls above (opts
 * supplies device_ptrs and stream; flags must be 0); d >= 1.  RRS_E_INVAL
 * also when the covariance is not positive definite (for example n <= d). */
rrs_status rrs_depth_mahalanobis(const double *X, int64_t n, int64_t d, const double *Z,
                                 int64_t m, double *depth, const rrs_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation inside a call):
 * rrs_depth_halfspace with the same arguments and results, except that
 *  - opts is required, with device_ptrs = 1: X, Z, depth, count and the
 *    optional poles / trace are device memory on the current device;
 *    flags must be 0 (capture the caller's stream instead of RRS_FLAG_GRAPH);
 *  - the call only enqueues its work on opts->stream and returns without
 *    waiting: the outputs are valid once that stream has passed the call;
 *  - every device buffer the call needs besides the caller's arrays comes from
 *    a static device array of RRS_NOALLOC_SCRATCH_MIB MiB that each device the
 *    library runs on holds until the process ends; the call makes no device
 *    or host allocation (no hipMalloc, hipFree, events or GEMM variant timing,
 *    and no query split over several streams).
 * The prepared data (about 8 n d bytes, plus 4 n (d + 16) for the bf16 form)
 * and the workspace of at least one query must fit the array; queries are
 * processed in batches that fit.  RRS_E_NOMEM when even one query does not
 * fit; RRS_E_INVAL as rrs_depth_halfspace, and for missing opts, host
 * pointers or non-zero flags.  All calls on one device share that device's
 * array: calls whose work overlaps on one device (several streams or
 * threads) race and must be serialised by the caller. */
#define RRS_NOALLOC_SCRATCH_MIB 256
rrs_status rrs_depth_halfspace_noalloc(const double *X, int64_t n, int64_t d,
                                       const double *Z, int64_t m, int64_t K,
                                       int32_t n_refine, double cap_shrink, uint64_t seed,
                                       double *depth, int64_t *count, const rrs_opts *opts);

/* Text of the last non-OK status returned on this thread ("" if none). */
const char *rrs_last_error(void);

/* Frees the workspace of every device.  Safe to call at any time between
 * calls. */
rrs_status rrs_release_workspace(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t rrs_version(void);

/* Per-kernel timing.  While enabled, every kernel launch of the depth calls
 * is bracketed by HIP events on the launch stream; each call reads them back
 * after synchronising its stream.  rrs_profile_enable(1) turns timing on and
 * clears the totals, rrs_profile_enable(0) turns it off.  rrs_profile_read
 * copies up to max_entries totals (one per kernel that ran) into out and
 * returns how many it wrote (out may be NULL to count them).  work_units is
 * the sum over launches of the units each launch processed: projections
 * (query x direction x point) for k_proj_f64, k_select and k_gemm,
 * coordinates for k_gen_dirs, directions for k_argmin_pole (0 for k_recheck,
 * which handles the pairs the matrix-core forms left uncertain). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
    double work_units;
} rrs_kernel_stat;

rrs_status rrs_profile_enable(int32_t on);
int32_t rrs_profile_read(rrs_kernel_stat *out, int32_t max_entries);

/* Event counters gathered while timing is on.  "select_fallback":
 * order-statistic pairs (median, MAD, MAD_+) resolved by the exact radix
 * fallback (counted on the device); "select_fast": the other selects, taken as
 * two per projection / APD column (an APD column without positive deviations
 * has one); "recheck_pairs": (query,
 * direction, point) projections the matrix-core forms recomputed in binary64;
 * "gemm_pairs": projections the halfspace sign GEMM evaluated (the others
 * were decided by the cap bound); "shared_full", "shared_median",
 * "shared_none": streamed APD columns whose shared passes served the whole
 * column, only its median, or nothing (the rest then took the separate
 * selects).
 * Returns 0 and writes *value, or -1 for an unknown name or NULL pointer. */
int32_t rrs_profile_counter(const char *name, double *value);

/* ------------------------------------------------------------------------
 * Serving: resident data sets and continuously batched requests.
 *
 * A context owns a slice of one device's memory (hbm_budget bytes, taken at
 * creation and sub-allocated by the library), `slots` HIP streams and one
 * scheduler thread.  Data sets are copied into the context once and stay
 * resident until released.  rrs_submit copies the queries and returns at
 * once; the scheduler admits pending requests in arrival order whenever a
 * slot and enough of the budget are free (a request that does not fit yet is
 * passed over by smaller later ones, at most 8 times, then admission waits
 * for it), and each admitted request runs on its own stream, overlapping on
 * the device with the others.  A request's result depends only on its own
 * arguments (data set, queries, query_offset, K, n_refine, cap_shrink, seed,
 * notion, precision): never on the other requests in flight.
 * ------------------------------------------------------------------------ */
typedef struct rrs_ctx rrs_ctx;
typedef struct rrs_dataset rrs_dataset;
typedef struct rrs_request rrs_request;

typedef struct {
    int32_t device;          /* HIP device ordinal */
    int32_t slots;           /* requests running at once (one stream each); 0: 4 */
    size_t hbm_budget;       /* device bytes for data sets and requests; 0: half
                                of the free memory */
    size_t request_ws_limit; /* workspace cap of one request (its queries are
                                batched to fit); 0: hbm_budget / (2 slots) */
} rrs_ctx_config;

/* Creates a context (cfg may be NULL for the defaults).  RRS_E_NOMEM when
 * the budget cannot be allocated, RRS_E_INVAL for a bad device or sizes. */
rrs_status rrs_ctx_create(const rrs_ctx_config *cfg, rrs_ctx **out);
/* Cancels pending requests (their rrs_wait returns RRS_E_CANCELLED), waits
 * for the running ones, releases every data set and the budget.  Request
 * handles stay valid for rrs_wait. */
rrs_status rrs_ctx_destroy(rrs_ctx *ctx);

/* Copies X (n x d row-major binary64, host memory) into the context and
 * prepares it; the caller keeps X.  RRS_E_NOMEM when it does not fit the
 * budget next to the resident data. */
rrs_status rrs_dataset_put(rrs_ctx *ctx, const double *X, int64_t n, int64_t d,
                           rrs_dataset **out);
/* Releases a data set; its memory returns to the budget once the requests
 * that use it have finished.  The handle is invalid afterwards. */
rrs_status rrs_dataset_release(rrs_ctx *ctx, rrs_dataset *ds);

/* Submits the depth (notion 0: halfspace, 1: projection, 2: asymmetric
 * projection) of the m queries Z (host, m x d, copied before return) on the
 * data set.  K, n_refine, cap_shrink, seed as for the synchronous calls;
 * opts (may be NULL) supplies precision, query_offset and workspace_limit --
 * device_ptrs, stream, poles and trace must be 0 / NULL.  RRS_E_NOMEM when
 * the request could never fit the budget; RRS_E_INVAL as the synchronous
 * calls. */
rrs_status rrs_submit(rrs_ctx *ctx, rrs_dataset *ds, int32_t notion, const double *Z, int64_t m,
                      int64_t K, int32_t n_refine, double cap_shrink, uint64_t seed,
                      const rrs_opts *opts, rrs_request **out);

/* Timestamps of a request in seconds of the host's monotonic clock
 * (CLOCK_MONOTONIC): submitted, admitted to a slot, result in host memory. */
typedef struct {
    double submit_s, admit_s, done_s;
    int64_t projections;     /* m x n_refine x ceil(K / n_refine) x n */
    size_t bytes;            /* device memory the request held while running */
} rrs_request_info;

/* Waits up to timeout_s seconds (< 0: no limit) for the request.  On
 * completion writes depth [m] (and count [m] for halfspace when count is not
 * NULL, and *info when info is not NULL), frees the request and returns its
 * status; on time-out returns RRS_E_BUSY and the handle stays valid. */
rrs_status rrs_wait(rrs_request *req, double timeout_s, double *depth, int64_t *count,
                    rrs_request_info *info);

typedef struct {
    int64_t pending, running, completed, failed;
    int64_t datasets;
    size_t bytes_in_use, bytes_peak, budget;
} rrs_ctx_stats;
rrs_status rrs_ctx_get_stats(rrs_ctx *ctx, rrs_ctx_stats *out);

/* Diagnostic for parity checks of the direction generator (step a1 alone):
 * writes the m_dir directions of refinement l (1-based) for the query whose
 * stream index is q, generated on the device exactly as inside the depth
 * calls, with cap scale phi = cap_shrink^(l-1) and pole p (both ignored for
 * l == 1).  pole: host [d]; out: host [m_dir x d], row-major.  Returns
 * RRS_E_INVAL for d < 2, m_dir < 1, l < 1 or NULL pointers. */
rrs_status rrs_debug_directions(int64_t d, int64_t m_dir, int32_t l, double phi, uint64_t seed,
                                uint64_t q, const double *pole, double *out);

#ifdef __cplusplus
}
#endif

#endif /* RRS_H */
