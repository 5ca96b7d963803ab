/*
 * geolik — exact Gaussian log-likelihood of a Matérn random field on one
 * AMD Instinct MI355X (gfx950), after ExaGeoStat (Abdulah et al., arXiv
 * 1708.02835).
 *
 * C ABI.  All pointers are DEVICE pointers (HIP global memory on the
 * context's device) unless the name ends in `_h` (host memory).  `stream` is
 * a `hipStream_t` passed as `void*` (NULL = the legacy default stream).  Every
 * vector is float64, contiguous, and owned by the caller unless stated.
 *
 * Return value of every `int` function: a gl_status.  Negative values are
 * usage or system errors (nothing was computed, or the result is unusable);
 * positive values are numerical outcomes.
 *
 * Threading: the direct calls (matern_generate, loglik_eval, krige_predict,
 * synth_generate) are stream-ordered and may not be called concurrently on
 * one context.  The lq_* request-queue calls are thread-safe.
 */
#ifndef GEOLIK_H
#define GEOLIK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gl_context gl_context;
typedef struct gl_factor gl_factor;
typedef struct lq_queue lq_queue;

/* Matérn parameters, Sec. 2.2 Eq. (2): variance θ1 > 0, range θ2 > 0,
 * smoothness θ3 > 0 (at most 50). */
typedef struct {
    double theta1;
    double theta2;
    double theta3;
} gl_theta;

typedef enum {
    GL_OK = 0,
    GL_NOT_SPD = 1,     /* Σ(θ) is not numerically positive definite; see gl_result.info */
    GL_EINVAL = -1,     /* bad argument (θ_i <= 0, n < 1, NULL pointer, bad option) */
    GL_ENOMEM = -2,     /* device allocation failed or the HBM budget is exceeded */
    GL_EHIP = -3,       /* a HIP runtime call failed */
    GL_EBUSY = -4,      /* lq_poll: request still pending */
    GL_ECANCELED = -5,  /* request cancelled or queue destroyed */
    GL_ETIMEDOUT = -6,  /* lq_wait: timeout elapsed */
    GL_ENODEV = -7,     /* no usable gfx950 device */
    GL_EVICTED = -9,    /* a factor kept through the queue was released by its admission */
    GL_E2BIG = -10      /* loglik_eval_noalloc: the workspace exceeds GL_SCRATCH_BYTES */
} gl_status;

typedef enum {
    GL_FP64 = 0,        /* every tile and every update in binary64 */
    GL_MIXED_FP32 = 1,  /* off-band trailing updates in binary32 on MFMA */
    GL_MIXED_BF16 = 2,  /* off-band updates as split-bfloat16 products, fp32 accumulate */
    GL_MIXED_FP16 = 3   /* off-band updates as scaled split-binary16 products, fp32 accumulate */
} gl_precision;

/* Precision classes of the tiles in the mixed modes (gl_precision_stats). */
enum { GL_NCLASS = 7 };

/* Options of one likelihood evaluation.  Fill with gl_opts_default().
 *
 * Mixed precision (not in the paper): every tile stays stored in binary64 and
 * the diagonal tiles, POTRF, TRSM, the solve and log|Σ| stay binary64; the
 * trailing products of off-band tiles (i, j) run at a precision chosen from
 * the normalised tile norm ν_ij = ||Σ_ij||_F / sqrt(||Σ_ii||_F ||Σ_jj||_F):
 *   both modes:    binary64 when ν_ij > tol_64 (strongly correlated tiles,
 *                  whose Schur complements cancel most);
 *   GL_MIXED_FP32: FP32 products otherwise;
 *   GL_MIXED_BF16: bfloat16 products with FP32 accumulation, operands split
 *                  in three parts (about FP32 accuracy) when ν_ij > tol_hi,
 *                  two parts when tol_lo < ν_ij <= tol_hi, one part below;
 *   GL_MIXED_FP16: binary16 products with FP32 accumulation of operands
 *                  scaled by a power of two (|L_ik| <= sqrt(max(θ1, 1)) maps
 *                  below 2^14), split in two parts (products hh + hl + lh,
 *                  about 22 bits) when ν_ij > tol_lo, one part below; tol_hi
 *                  is not used.
 * Thresholds left negative (the default) are adaptive: with the accuracy
 * target ε (default 1e-4) and ρ = min_r L_rr² / θ1 over the first diagonal
 * tile (its binary64 POTRF runs before any off-band update; ρ is the smallest
 * conditional variance ratio of those locations, small when neighbours
 * explain most of a value and the Schur complements cancel), a class with
 * unit roundoff u is used for tile (i, j) only while ν_ij u <= ε ρ:
 * tol_64 = ε ρ / 2⁻²⁴, tol_hi = ε ρ / 2⁻¹⁶, tol_lo = ε ρ / 2⁻⁸ (FP32 and
 * BF16 modes); tol_64 = ε ρ / 2⁻²², tol_lo = ε ρ / 2⁻¹¹ (FP16 mode).
 * Tiles with i - j < band stay binary64.  The mixed modes keep FP32 running
 * sums of the updates, so they require θ1 <= 1e30 (GL_EINVAL otherwise).
 *
 * Distance (Sec. 2 and Sec. 7.4): metric GL_EUCLIDEAN uses r = ||s_i - s_j||
 * in the plane; GL_GREAT_CIRCLE reads x as longitude and y as latitude in
 * degrees and uses the great-circle distance on a sphere of the given radius
 * (haversine formula), in the radius' unit (θ2 in the same unit). */
enum { GL_EUCLIDEAN = 0, GL_GREAT_CIRCLE = 1 };

typedef struct {
    int32_t precision;   /* gl_precision */
    int32_t tile;        /* tile size b: 0 = automatic, else 128, 256, 384 or 512 */
    int32_t keep_factor; /* 1: return the Cholesky factor in gl_result.factor for kriging */
    int32_t band;        /* mixed modes: tiles with i - j < band stay binary64 (>= 1) */
    int32_t reorder;     /* -1: automatic (Morton order for the mixed modes, input order for
                            GL_FP64); 0: input order; 1: Morton order.  l(θ) does not depend
                            on the order; kept factors are in the order used. */
    int32_t metric;      /* GL_EUCLIDEAN (default) or GL_GREAT_CIRCLE */
    double tol_hi;       /* GL_MIXED_BF16: see above (negative: adaptive) */
    double tol_lo;       /* GL_MIXED_BF16 and GL_MIXED_FP16: see above (negative: adaptive) */
    double radius;       /* GL_GREAT_CIRCLE: sphere radius (> 0; default 6371, the Earth in km) */
    double tol_64;       /* mixed modes: see above (negative: adaptive) */
    double accuracy;     /* mixed modes: ε of the adaptive thresholds (negative: 1e-4) */
    int32_t ind_tiles;   /* 0: exact l(θ).  s >= 1: independent-blocks approximation (Sec. 6.8):
                            every tile outside the diagonal super tiles of s×s tiles is
                            annihilated, i.e. l is summed over blocks of s·b consecutive
                            locations (after reordering, if on), each factored on its own;
                            GL_FP64 only, no kept factor (krige_cv also takes it) */
    int32_t graph;       /* 1: GL_FP64 without a kept factor runs everything after staging the
                            inputs as a replayed hipGraph, captured on the first call for a
                            workspace geometry (n, tile) and distance and replayed while they
                            stay the same (θ is read from device memory); 0: direct launches */
    int32_t near_tiles;  /* schedule of the trailing updates (results change by rounding only).
                            GL_FP64 and the split-product classes of the mixed modes apply two
                            panels per pass (K = 2b) to the columns beyond the nearest ones: at
                            an even step k the next column and the nearest columns holding about
                            near_tiles tiles get panel k alone, the others get panels k and k+1
                            together at step k+1.  0: automatic, b tiles (GL_FP64) or
                            1536 (512/b)³ split-product tiles (mixed modes); > 0: that many */
    int32_t layout;      /* matern_generate only: GL_LAYOUT_DENSE (default) or
                            GL_LAYOUT_LOWER_TILES (see there) */
} gl_opts;

enum { GL_LAYOUT_DENSE = 0, GL_LAYOUT_LOWER_TILES = 1 };

/* Result of one likelihood evaluation, host memory. */
typedef struct {
    double loglik;      /* l(θ), Eq. (1); -INFINITY when status == GL_NOT_SPD */
    double logdet;      /* log|Σ(θ)| = 2 Σ log L_ii */
    double quad;        /* Zᵀ Σ(θ)⁻¹ Z = wᵀw, w = L⁻¹ Z */
    int64_t info;       /* 0, or the 1-based global column of the first non-positive pivot */
    int32_t status;     /* gl_status of the evaluation */
    int32_t tile;       /* tile size used */
    gl_factor *factor;  /* owned factor when keep_factor = 1 and status == GL_OK, else NULL */
} gl_result;

/* ------------------------------------------------------------ context ---- */

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the device
 * memory the library holds for factors and workspaces (0 = 90% of the free
 * memory at creation).  Errors: GL_EINVAL (out == NULL), GL_ENODEV, GL_EHIP. */
int gl_context_create(int device, size_t hbm_budget_bytes, gl_context **out);

/* Release every workspace, factor and dataset still held; queues still alive
 * are destroyed first (as lq_destroy: running requests finish, queued ones
 * are cancelled).  The caller must not use factors or queues of this context
 * afterwards. */
void gl_context_destroy(gl_context *ctx);

/* Fill *opts with defaults: FP64, automatic tile, no factor kept, band 2,
 * automatic order, mode-default thresholds (-1), automatic near_tiles (0). */
void gl_opts_default(gl_opts *opts);

/* Static English description of a gl_status value. */
const char *gl_status_string(int status);

/* Tile size b a likelihood evaluation of size n uses for the requested tile
 * (0 = automatic: 128 up to n = 3,000, 256 up to 24,000, 512 beyond).
 * Returns b, or GL_EINVAL for n < 1 or a tile other than 0, 128, 256, 384,
 * 512.  Host arithmetic only. */
int32_t gl_pick_tile(int64_t n, int32_t tile);

/* Device bytes a likelihood evaluation of size n at tile b holds
 * (packed lower tiles plus vectors), b = 0 meaning the automatic choice. */
size_t gl_footprint_bytes(int64_t n, int32_t tile, int32_t precision);

/* The same footprint split into the workspace's three device allocations:
 * packed lower tiles, vectors (padded locations and measurements, per-tile
 * sums, inverses of the 64×64 diagonal blocks, result words, sort keys) and
 * the mixed-precision side buffer (0 for GL_FP64), in bytes.  A workspace is
 * reallocated only where a size grows.  Pure host arithmetic: needs no device.
 * Errors: GL_EINVAL for n < 1 or a bad tile or precision.  Any output may be
 * NULL. */
int gl_workspace_layout(int64_t n, int32_t tile, int32_t precision, size_t *tiles_h, size_t *vecs_h,
                        size_t *mix_h);

/* --------------------------------------------------------- operations ---- */

/*
 * Matérn covariance between point sets 1 and 2, Sec. 2.2 Eq. (2) with the
 * distance of opts->metric (NULL opts: Euclidean, dense layout; other fields
 * ignored except layout and tile) (genDistanceMatrix + genCovMatrix of
 * Alg. 1-3, the distance matrix is never stored).  r == 0 gives θ1.
 * opts->layout:
 *   GL_LAYOUT_DENSE: column-major n1×n2, out[i + j*ld], ld >= n1.
 *   GL_LAYOUT_LOWER_TILES: Σ of set 1 with itself (x2, y2 NULL, or equal to
 *     x1, y1 with n2 == n1; ld ignored) in the packed lower-tile storage the
 *     likelihood factors: tile size b = opts->tile (0: the automatic choice of
 *     loglik_eval), NT = ceil(n1 / b) tile rows, tile (i, j), i >= j, a b×b
 *     column-major block at out + (i(i+1)/2 + j)·b², NT(NT+1)/2·b² doubles in
 *     all (gl_workspace_layout's tiles bytes / 8).  Diagonal tiles are written
 *     in full (both triangles); rows and columns beyond n1 are padding, 1 on
 *     the diagonal and 0 elsewhere.
 * The caller owns out.
 * Errors: GL_EINVAL for n1 < 1, NULL pointers, bad θ, a bad metric/radius,
 * layout or tile, and for the dense layout n2 < 1 or ld < n1.
 */
int matern_generate(gl_context *ctx, const double *x1, const double *y1, int64_t n1,
                    const double *x2, const double *y2, int64_t n2, gl_theta theta,
                    const gl_opts *opts, double *out, int64_t ld, void *stream);

/*
 * l(θ) = -n/2 log 2π - ½ log|Σ(θ)| - ½ Zᵀ Σ(θ)⁻¹ Z, Sec. 2 Eq. (1), computed
 * as in Alg. 2: Σ(θ) in packed lower tiles, tiled Cholesky Σ = L Lᵀ,
 * forward solve w = L⁻¹ Z, log|Σ| = 2 Σ log L_ii, Zᵀ Σ⁻¹ Z = wᵀw.
 * Inputs x, y, z: n locations and measurements (device).  opts may be NULL
 * (defaults).  The call is synchronous with respect to `stream`: it returns
 * after the result is in *res_h.  Return value equals res_h->status.
 * With keep_factor = 1 and status GL_OK, res_h->factor owns device memory
 * until gl_factor_release (it counts against the HBM budget).
 */
int loglik_eval(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
                gl_theta theta, const gl_opts *opts, gl_result *res_h, void *stream);

/*
 * loglik_eval for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, hosts that forbid hipMalloc): the same
 * binary64 computation and kernels as loglik_eval, bit-identical results, but
 * the workspace lives in a static device array of GL_SCRATCH_BYTES per device
 * (held until the process ends) and the call allocates nothing, on the device
 * or the host.  The context must have been created beforehand (that is where
 * the array's device address is looked up).
 * Limits: precision GL_FP64, keep_factor = 0, graph = 0, ind_tiles = 0
 * (GL_EINVAL otherwise); the workspace of (n, tile) — gl_workspace_layout's
 * tiles rounded up to 256 bytes, plus its vectors — must fit GL_SCRATCH_BYTES
 * (GL_E2BIG otherwise, nothing launched): n <= 4,096 at every tile size.
 * Kernel timing (gl_profile_enable) does not cover this call.
 * Every call on one device shares that device's array, whatever the context:
 * calls that overlap on one device race, and must be ordered by the caller.
 * Synchronous with respect to `stream` like loglik_eval; return value equals
 * res_h->status.
 */
#define GL_SCRATCH_BYTES ((size_t)96 << 20)
int loglik_eval_noalloc(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
                        gl_theta theta, const gl_opts *opts, gl_result *res_h, void *stream);

/*
 * Kriging, Sec. 2.3 Eq. (5) and Alg. 3: Z1 = Σ12 Σ22⁻¹ Z2 at m new locations,
 * reusing the factor L of a previous loglik_eval (keep_factor = 1) and its
 * forward solution w: X = L⁻ᵀ w, then Z1_k = Σ_j C(||s_new,k - s_j||) X_j with
 * Σ12 generated on the fly and never stored, with the factor's distance.
 * Output znew: m doubles (device, caller-owned).
 * var (may be NULL): the prediction variances, the diagonal of the
 * conditional covariance of Eq. (4), var_k = θ1 - ||L⁻¹ σ_k||² with σ_k the
 * covariances between new location k and the n observed ones; the m
 * right-hand sides are solved together on the matrix cores, 512 at a time.
 * Asynchronous on `stream`.
 * Errors: GL_EINVAL for a NULL or unknown factor, m < 1 or NULL pointers;
 * GL_ENOMEM when the variance workspace (n·min(m, 512) doubles) does not fit;
 * GL_EVICTED for a queue-kept factor whose memory the queue released.
 */
int krige_predict(gl_context *ctx, gl_factor *factor, const double *xnew, const double *ynew,
                  int64_t m, double *znew, double *var, void *stream);

/*
 * k-fold cross-validation of kriging (Sec. 7.3: the prediction MSE
 * of held-out measurements).  fold_h (host, n values in
 * 0..k-1, drawn by the caller) assigns each location to a fold; for each fold
 * f the locations outside it are factored (loglik_eval with keep_factor, the
 * other opts as given), the fold's measurements are predicted by Eq. (5), and
 * mse_h[f] (host, k doubles) receives the mean squared prediction error over
 * the fold.  With opts->ind_tiles = s >= 1 the prediction uses the IND
 * approximation (Sec. 6.8; the exact-versus-IND prediction comparison of the
 * paper's experiments) of the covariance of all n locations: blocks of s·b
 * consecutive locations in input order (b the tile size) are independent
 * fields, so each held-out value is predicted by Eq. (5) from the observed
 * values of its own block (0 when the block observes nothing); reorder = 1 is
 * rejected there.  Synchronous with respect to `stream`.
 * pred (device, n doubles, may be NULL): pred[i] receives the prediction of
 * location i from the folds other than its own, in input order (the values
 * the MSE of its fold is taken over); the entries of a fold whose Σ was not
 * positive definite are left untouched.
 * Returns GL_OK; GL_NOT_SPD when some fold's Σ was not positive definite (its
 * mse_h is NaN, the other folds are still computed); GL_EINVAL for k < 2, a
 * fold id out of range, an empty fold or a fold holding every location.
 */
int krige_cv(gl_context *ctx, const double *x, const double *y, const double *z, int64_t n,
             gl_theta theta, const gl_opts *opts, const int32_t *fold_h, int32_t k, double *mse_h,
             double *pred, void *stream);

/* Release a factor returned by loglik_eval or through the request queue
 * (also one the queue has evicted). */
int gl_factor_release(gl_context *ctx, gl_factor *factor);

/* Copy the lower-triangular factor L of `factor` into a dense column-major
 * n×n array (device, ld >= n) with a zero strict upper triangle, in the
 * order the factorisation used (input order unless reordering was on). */
int gl_factor_to_dense(gl_context *ctx, gl_factor *factor, double *out, int64_t ld, void *stream);

/* Order n and tile size of a factor (either output may be NULL). */
int gl_factor_shape(const gl_factor *factor, int64_t *n, int32_t *tile);

/*
 * Synthetic measurements, Sec. 6.4 Alg. 1: Σ(θ) = L Lᵀ (tiled Cholesky) and
 * Z = L e.  Inputs x, y, e: n values each (device).  Output z: n doubles.
 * opts (may be NULL): tile and distance; precision must be GL_FP64, other
 * fields are ignored.  Synchronous with respect to `stream`; *info_h (may be
 * NULL) receives the Cholesky info.  Returns GL_OK or GL_NOT_SPD.
 */
int synth_generate(gl_context *ctx, const double *x, const double *y, const double *e,
                   int64_t n, gl_theta theta, const gl_opts *opts, double *z, int64_t *info_h,
                   void *stream);

/* ------------------------------------------------------------ serving ---- */

/* Register a dataset (locations and measurements) for the request queue.  The
 * library copies x, y, z (device pointers) into memory it owns; the caller may
 * free its buffers when the call returns.  *ds_h receives the dataset id. */
int gl_dataset_register(gl_context *ctx, const double *x, const double *y, const double *z,
                        int64_t n, uint64_t *ds_h);

/* Drop a dataset.  Pending requests on it are cancelled. */
int gl_dataset_release(gl_context *ctx, uint64_t ds);

/* Queue configuration.  Fill with lq_config_default(). */
typedef struct {
    int32_t max_inflight;    /* requests resident on the device at once (1..64) */
    int32_t streams;         /* requests run one at a time per stream outside the fused
                                launches; this many such streams (1..8), each created
                                when its first request arrives (the fused launches use
                                two streams of their own) */
    int32_t batch_small;     /* 1: FP64 requests with n <= small_n (tile 0 or 256, no
                                reordering) advance together through fused launches,
                                one factorisation step per launch, tile 256 */
    int32_t small_n;         /* size limit of the fused path */
    size_t hbm_budget_bytes; /* admission budget for resident work (0 = the context's) */
} lq_config;

void lq_config_default(lq_config *cfg);

/* Start a scheduler thread serving likelihood requests of `ctx`. */
int lq_create(gl_context *ctx, const lq_config *cfg, lq_queue **q_h);

/* Enqueue l(θ) on dataset ds; thread-safe.  *ticket_h identifies the request.
 * opts may be NULL (defaults; graph is ignored by the queue).
 * keep_factor = 1: a successful request's result carries its factor (for
 * krige_predict, Alg. 3), owned by the caller until gl_factor_release.  Its
 * device memory counts against the queue's HBM budget; when admitting a
 * request needs room, the queue first drops idle workspaces, then releases
 * the memory of the factors it handed out, least recently used first (a
 * kriging call marks a use), waiting for kernels still reading them.  Calls on
 * a released factor return GL_EVICTED; its handle stays valid until
 * gl_factor_release.  Factors outlive the queue (lq_destroy makes them
 * permanent).
 * Errors: GL_EINVAL for an unknown dataset, bad θ or options, or ind_tiles != 0
 * (the independent-blocks approximation is a direct call only); GL_ECANCELED
 * once the queue is being destroyed. */
int lq_submit(lq_queue *q, uint64_t ds, gl_theta theta, const gl_opts *opts, uint64_t *ticket_h);

/* Non-blocking: GL_EBUSY while pending, else copies the result and retires
 * the ticket (returns the request's status). */
int lq_poll(lq_queue *q, uint64_t ticket, gl_result *res_h);

/* Blocking with a timeout in microseconds (< 0 = forever): GL_ETIMEDOUT or
 * the request's status; a delivered result retires the ticket. */
int lq_wait(lq_queue *q, uint64_t ticket, gl_result *res_h, int64_t timeout_us);

/* Cancel a request that has not started on the device. GL_OK if cancelled,
 * GL_EBUSY if it is already running or done. */
int lq_cancel(lq_queue *q, uint64_t ticket);

/* Counters since creation: completed requests, peak resident bytes, peak
 * requests resident at once, fused launches issued. Any pointer may be NULL. */
int lq_stats(lq_queue *q, uint64_t *completed, size_t *peak_bytes, int32_t *peak_inflight,
             uint64_t *fused_launches);

/* Overhead of the fused path since creation: ticks issued, host time spent
 * building and enqueuing them (µs, summed), device time from a tick's first
 * to its last command (ms, summed over retired ticks; the two cohorts overlap,
 * so the sum may exceed the wall time) and device idle time between
 * consecutive ticks of one cohort (ms, summed).  Any pointer may be NULL. */
int lq_tick_stats(lq_queue *q, uint64_t *ticks, double *host_us, double *device_ms, double *gap_ms);

/* Stop the scheduler: requests not yet started are cancelled, running ones are
 * drained, then the thread exits and the queue is freed. */
int lq_destroy(lq_queue *q);

/* Morton (Z-order) permutation of n locations: perm[i] (device, n int64) is
 * the input index of position i.  Coordinates are quantised to 16 bits over
 * their bounding box; ties are broken by the input index, so the permutation
 * is unique.  This is the order the mixed modes factor in. */
int gl_morton_order(gl_context *ctx, const double *x, const double *y, int64_t n, int64_t *perm,
                    void *stream);

/* --------------------------------------------------------- diagnostics ---- */

/* Precision map of the last mixed-precision loglik_eval on this context:
 * tiles per class and work per class (Σ over tiles of the trailing updates
 * they receive), classes 0 FP64, 1 FP32, 2 BF16x6, 3 BF16x3, 4 BF16,
 * 5 FP16x3 (two parts), 6 FP16 (GL_NCLASS = 7 values each), and
 * thresholds_h = {ρ, tol_64, tol_hi, tol_lo} as used (4 values).
 * Any pointer may be NULL. */
int gl_precision_stats(gl_context *ctx, int64_t *tiles_h, double *work_h, double *thresholds_h);

/* Runs a built-in device self-check `which` and writes up to `cap` doubles of
 * output to out_h: 0 = the lane layout of the FP64 16x16x4 matrix-core
 * product (256 values), 1 = the same for FP32 16x16x4, 2 = BF16 16x16x32,
 * 3 = FP16 16x16x32. */
int gl_selftest(gl_context *ctx, int32_t which, double *out_h, int64_t cap);

/* Kernel timing by phase of Alg. 2.  While enabled, kernel launches of the
 * direct calls are bracketed by HIP events on the stream they run on: on = 1
 * the trailing updates only (the dominant kernel family), on = 2 every phase
 * below; 0 switches timing off.  In the mixed-precision modes only the
 * trailing updates are timed, by precision class (the GL_PHASE_MIXED_*
 * phases: one per class of gl_precision_stats, binary64 to one-part
 * binary16; a mixed call whose tiles all stay binary64 runs, and is timed
 * as, the binary64 schedule).  Phases run on three streams (critical path, lookahead and
 * forward solve), so summed durations may exceed the wall time. */
enum {
    GL_PHASE_GEN = 0,        /* Σ(θ) tile generation (Eq. 2) */
    GL_PHASE_POTRF = 1,      /* diagonal-tile factorisations (b³/3 flops each) */
    GL_PHASE_TRSM = 2,       /* panel solves (b³ flops per panel tile) */
    GL_PHASE_SOLVE = 3,      /* forward solve w = L⁻¹Z (2b² flops per tile) */
    GL_PHASE_TRAIL_CRIT = 4, /* trailing update of the next tile column, critical path */
    GL_PHASE_TRAIL_BULK = 5, /* trailing update of the other columns, lookahead stream */
    GL_PHASE_REDUCE = 6,     /* log|Σ|, ZᵀΣ⁻¹Z and l(θ) (Eq. 1) */
    GL_PHASE_TRAIL_PAIR = 7, /* trailing updates of the far columns by two panels in one pass
                                (lookahead stream; see gl_opts.near_tiles) */
    GL_PHASE_MIXED_FP64 = 8,   /* mixed modes: trailing updates of the binary64 class */
    GL_PHASE_MIXED_FP32 = 9,   /* ... the FP32 class */
    GL_PHASE_MIXED_BF16X6 = 10, /* ... three bfloat16 parts, six products */
    GL_PHASE_MIXED_BF16X3 = 11, /* ... two bfloat16 parts, three products */
    GL_PHASE_MIXED_BF16 = 12,   /* ... one bfloat16 part */
    GL_PHASE_MIXED_FP16X3 = 13, /* ... two scaled binary16 parts, three products */
    GL_PHASE_MIXED_FP16 = 14,   /* ... one scaled binary16 part */
    GL_NPHASE = 15
};
int gl_profile_enable(gl_context *ctx, int32_t on);
/* Synchronises the device and returns, per phase (GL_NPHASE values each; any
 * pointer may be NULL), the summed launch durations (ms), the algorithmic
 * flops of those launches (trailing: 2b³ per off-diagonal tile update, b²(b+1)
 * per diagonal tile update, whatever the precision class; generation and
 * reduction: 0) and the launch count since the last read, then resets them. */
int gl_profile_phases(gl_context *ctx, double *ms_h, double *flops_h, int64_t *launches_h);
/* The same for the three binary64 trailing phases together (one value each). */
int gl_profile_read(gl_context *ctx, double *ms_h, double *flops_h, int64_t *launches_h);

#ifdef __cplusplus
}
#endif
#endif /* GEOLIK_H */
