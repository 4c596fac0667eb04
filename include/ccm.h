/*
 * ccm.h -- C ABI of libccm: batched simplex cross-map prediction, the hot
 * path of convergent cross mapping (CCM), on one AMD Instinct MI355X (gfx950).
 *
 * What a call computes (paper: Pu, Duan & Osgood, "Parallelizing Convergent
 * Cross Mapping Using Apache Spark"):
 *   For series X and Y, embedding dimension E and delay tau (Introduction:
 *   the parameters r, tau, E, L), build the lagged-coordinate shadow manifold
 *   of the library series; for each library size L draw r random library
 *   subsamples (Introduction; Section 3.1: the input record is a pair of
 *   subsamples of length L plus (tau, E)); for every query point find its E+1
 *   nearest library vectors by brute force (Section 3.2: distances to all
 *   lagged-coordinate vectors, sorted, first E+1); predict the other series
 *   by simplex projection (Section 2.1) with weights exp(-d_i / d_1); and
 *   report the Pearson correlation of observed and predicted values as the
 *   prediction skill (Section 2.1), in both directions (Introduction).  The
 *   output is one skill per realization: the "sequence of prediction skills"
 *   of Section 3.1.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - embedded point i (0-based) is at time t_i = i + (E-1) tau, coordinate
 *     k = S[t_i - k tau]; the predicted value is the target at t_i;
 *     N_e = N - (E-1) tau embedded points;
 *   - squared distances are binary32: both series are rounded to float, then
 *     acc = fma(d_k, d_k, acc), k = 0..E-1 from +0, d_k = q_k - p_k in float;
 *     neighbours are the first E+1 candidates in (d2, index) order, so ties
 *     go to the lower time index;
 *   - d_m = sqrt(d2_m) in double; w_m proportional to exp(-d_m / d_1); when
 *     d_1 = 0 the weight is shared equally by the zero-distance neighbours;
 *   - libraries are drawn without replacement by selection sampling driven
 *     by SplitMix64; the draw of realization r_index depends only on
 *     (seed, E, tau, L_eff, r_index), so both directions (and every series
 *     of ccm_matrix) share it;
 *   - L above N_e is clamped to L_eff = N_e (then every realization is the
 *     same full library);
 *   - rho is NaN when the observed or the predicted values are constant.
 *
 * Ownership: every pointer argument is borrowed for the duration of the call
 * (host pointers) or until the work queued on the given stream has run
 * (device pointers).  Outputs are caller-allocated.  The context owns all
 * device memory it allocates.
 *
 * Threading: a context serialises its calls internally; use one context per
 * host thread for concurrency.
 *
 * Errors: every function returns a ccm_status.  CCM_E_INVAL for a null
 * pointer, N < 2, E outside [1, 10], tau < 1, N_e < E + 2, any L < E + 2,
 * an L_eff too small for the exclusion window (L_eff < E + 2 + 2w), r < 1,
 * nL < 1, a non-finite input value or |value| > 1e17 (which keeps every
 * binary32 squared distance finite).  CCM_E_NOMEM when device memory cannot
 * be allocated, CCM_E_DEVICE for any failing HIP call; ccm_last_error()
 * returns the message.  No C++ exception crosses this interface.
 */
#ifndef CCM_H
#define CCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CCM_OK = 0,
  CCM_E_INVAL = -1,
  CCM_E_NOMEM = -2,
  CCM_E_DEVICE = -3,
  CCM_E_BUSY = -4,
  CCM_E_NOTFOUND = -5,
  CCM_E_TIMEOUT = -6
} ccm_status;

typedef struct ccm_ctx ccm_ctx;

/* Options (NULL means all defaults). */
typedef struct {
  /* 0: drop the query point itself from its candidates (default);
     -1: keep it; w > 0: drop every candidate j with |j - i| <= w. */
  int32_t exclusion_radius;
  /* 0: predict at every embedded point (default); 1: at the library points. */
  int32_t query_set;
  /* CCM_FLAG_* bits. */
  uint32_t flags;
} ccm_opts;

/* One kernel launch per realization instead of one batched launch (the
   unbatched baseline the batched form is compared against). */
#define CCM_FLAG_PLAIN 1u
/* Issue the batched launches directly instead of replaying a captured
   HIP graph. */
#define CCM_FLAG_NO_GRAPH 2u
/* Cross-map kernel as a persistent grid pulling work items from an atomic
   queue (default: one workgroup per work item, longest first). */
#define CCM_FLAG_PERSISTENT 4u
/* Distance indexing table (Section 3.2): before the cross map, build for
   every library embedding that needs it a table whose row i lists the
   first CCM_TABLE_WIDTH embedded points in ascending (d2, index) order
   from point i, and find each query's E+1 neighbours by walking its row
   until E+1 library members (not excluded) are seen.  Used for the
   realizations whose expected walk is short (large libraries); the others,
   and any wavefront whose walk runs off the end of its rows, scan by brute
   force.  Neighbours, predictions and rho are bitwise identical to the
   brute-force path.  Costs n_e * CCM_TABLE_WIDTH * 4 bytes of device memory
   per table.  Honoured by the served form too (ccm_submit). */
#define CCM_FLAG_TABLE 8u
#define CCM_TABLE_WIDTH 1024
/* Nested libraries (an option of this library, not of the paper): the
   library of (E, tau, L, r) is the first L_eff points of one uniformly
   random ordering of the embedded points per (E, tau, r) -- a forward
   Fisher-Yates shuffle driven by the SplitMix64 stream keyed by
   (seed, E, tau, r) -- so the libraries of one r grow by inclusion with L.
   Each query then scans the largest library once, in segments, taking its
   E+1 neighbours at every library size: the cross map costs
   N_e * max(L_eff) pairs per (E, tau, r, direction) instead of
   N_e * sum(L_eff).  The rho values differ from the default draws (the
   libraries are correlated across L).  ccm and ccm_sweep (and their device
   forms) only, with query_set 0; not with CCM_FLAG_TABLE, CCM_FLAG_PLAIN or
   CCM_FLAG_SHARED_E (CCM_E_INVAL). */
#define CCM_FLAG_NESTED 16u
/* E-sweep sharing (an option of this library, not of the paper): for each
   tau, every E of the call uses the points that E_max (the largest E
   listed) can embed -- N_c = N - (E_max-1) tau of them, point c at time
   c + (E_max-1) tau, its first E lag coordinates as E's point -- and one
   library per (tau, L, r) drawn over those N_c points by the SplitMix64
   stream keyed by (seed, 0, tau, L_eff, r).  Each E is then the default
   cross map of the series shifted by (E_max-E) tau, and one scan per
   (tau, L, r, direction) computes every E's neighbours: the binary32
   distance after E coordinates is E's d2.  The rho values differ from the
   default draws (fewer points for E < E_max, other libraries).  ccm and
   ccm_sweep (and their device forms) only, with query_set 0; not with
   CCM_FLAG_TABLE, CCM_FLAG_NESTED or CCM_FLAG_PLAIN (CCM_E_INVAL). */
#define CCM_FLAG_SHARED_E 32u

/* Create a context on HIP device `device`.  *out receives the handle. */
ccm_status ccm_create(int device, ccm_ctx **out);
/* Release the context and all device memory it owns (NULL is a no-op). */
void ccm_destroy(ccm_ctx *ctx);
/* Message of the last failing call on this context ("" if none).  The
   string stays valid until the next call on the context. */
const char *ccm_last_error(const ccm_ctx *ctx);

/*
 * Memory bound of the batched calls (ccm, ccm_sweep, ccm_matrix and their
 * device forms).  Each realization needs its drawn library (the paper's
 * subsample, Section 3.1) and that library laid out for the scan: about
 * L_eff * (E + 2) * 4 bytes of device memory (nested libraries: also N_e * 4
 * per ordering).  The realizations of a call run in waves whose libraries
 * together fit `bytes`: all realizations of one E in one wave when they
 * fit, consecutive E merged while they fit, one E split over several waves
 * when it alone does not fit (at least one realization per wave).  The
 * results do not depend on the bound; other buffers of a call (series,
 * embeddings, visiting orders, per-tile moments) are not counted.  bytes = 0
 * restores the default, min(8 GiB, device memory / 8) and at least 1 GiB.
 * The bound applies to calls made after it is set.
 */
ccm_status ccm_set_wave_limit(ccm_ctx *ctx, uint64_t bytes);

/*
 * Cross map in both directions for one (E, tau): Introduction and
 * Sections 2.1, 3.1, 3.2.
 *   X, Y        host double[N] series
 *   L           host int64[nL] library sizes
 *   r           realizations (random libraries) per L
 *   seed        sampler seed
 *   rho_X_from_MY  host double[nL][r]: skill of predicting X from the
 *                  manifold of Y (high when X drives Y)
 *   rho_Y_from_MX  host double[nL][r]
 *   L_eff       host int64[nL] (nullable): clamped library sizes
 */
ccm_status ccm(ccm_ctx *ctx, const double *X, const double *Y, int64_t N,
               int32_t E, int32_t tau, const int64_t *L, int32_t nL, int32_t r,
               uint64_t seed, const ccm_opts *opts, double *rho_X_from_MY,
               double *rho_Y_from_MX, int64_t *L_eff);

/*
 * Parameter sweep (Introduction: results are sensitive to E, tau and L and
 * are explored over a range of settings; Section 3.3 runs the settings
 * concurrently).  All realizations of every (E, tau, L, r) run as one
 * batched launch per E.
 *   E, tau      host int32[nE], int32[ntau]
 *   rho         host double[2][nE][ntau][nL][r]; [0] = X from M_Y,
 *               [1] = Y from M_X
 */
ccm_status ccm_sweep(ccm_ctx *ctx, const double *X, const double *Y,
                     int64_t N, const int32_t *E, int32_t nE,
                     const int32_t *tau, int32_t ntau, const int64_t *L,
                     int32_t nL, int32_t r, uint64_t seed,
                     const ccm_opts *opts, double *rho);

/*
 * Causal matrix over M series (Introduction: unidirectional and
 * bidirectional links between variables; every ordered pair is a
 * cross map).  One neighbour search on the manifold of series a serves the
 * prediction of every other series b (the library draw does not depend on
 * the series).
 *   S           host double[M][N], row-major
 *   rho         host double[M][M][nL][r]: rho[a][b] is the skill of
 *               predicting series b from the manifold of series a (high when
 *               b drives a); the diagonal is NaN
 * Requires M >= 2 and (M rounded up to even) * N <= 2^29 (the targets are
 * kept as one time-major FP64 table within 4 GiB), else CCM_E_INVAL; other
 * rules as for ccm().
 */
ccm_status ccm_matrix(ccm_ctx *ctx, const double *S, int32_t M, int64_t N,
                      int32_t E, int32_t tau, const int64_t *L, int32_t nL,
                      int32_t r, uint64_t seed, const ccm_opts *opts,
                      double *rho);

/*
 * Device-pointer forms: X, Y (double[N]), S (double[M][N]) and rho are
 * device pointers, the other arrays are host pointers; the work is queued on `stream` (a
 * hipStream_t; NULL = the null stream) and the call returns without waiting.
 * Output layouts as above.
 */
ccm_status ccm_dev(ccm_ctx *ctx, const double *X, const double *Y, int64_t N,
                   int32_t E, int32_t tau, const int64_t *L, int32_t nL,
                   int32_t r, uint64_t seed, const ccm_opts *opts,
                   double *rho_X_from_MY, double *rho_Y_from_MX,
                   int64_t *L_eff, void *stream);
ccm_status ccm_sweep_dev(ccm_ctx *ctx, const double *X, const double *Y,
                         int64_t N, const int32_t *E, int32_t nE,
                         const int32_t *tau, int32_t ntau, const int64_t *L,
                         int32_t nL, int32_t r, uint64_t seed,
                         const ccm_opts *opts, double *rho, void *stream);
ccm_status ccm_matrix_dev(ccm_ctx *ctx, const double *S, int32_t M, int64_t N,
                          int32_t E, int32_t tau, const int64_t *L, int32_t nL,
                          int32_t r, uint64_t seed, const ccm_opts *opts,
                          double *rho, void *stream);

/*
 * No-allocation form of ccm_dev, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, computation and results (bit for bit)
 * as ccm_dev with no flags; it calls no hipMalloc or hipFree: every device
 * buffer of the call -- descriptors, series copies, embeddings, visiting
 * orders, libraries, per-tile moments, rho -- is a range of one static
 * workspace of CCM_NOALLOC_WORKSPACE_BYTES per device, held from the first
 * context on that device until the process ends.  The descriptors are
 * copied from host memory of the call with hipMemcpyAsync (pageable: staged
 * before the call returns); the rest is queued on `stream` as in ccm_dev.
 * CCM_E_NOMEM, with a message, when the call needs more than the workspace
 * holds (about 16 MB for N = 1000, E = 2, ten L to 1000, r = 100);
 * CCM_E_INVAL for flags other than CCM_FLAG_NO_GRAPH.  Every call on one
 * device uses the same workspace and leaves its contents there: calls that
 * overlap on one device (different streams, contexts or host threads
 * without ordering between them) race; calls ordered on one stream do not.
 */
#define CCM_NOALLOC_WORKSPACE_BYTES (64ull << 20)
ccm_status ccm_dev_noalloc(ccm_ctx *ctx, const double *X, const double *Y, int64_t N,
                           int32_t E, int32_t tau, const int64_t *L, int32_t nL,
                           int32_t r, uint64_t seed, const ccm_opts *opts,
                           double *rho_X_from_MY, double *rho_Y_from_MX,
                           int64_t *L_eff, void *stream);

/*
 * Served form: continuous batching of independent cross-map jobs (paper
 * Section 3.3: several (L, tau, E) pipelines run concurrently instead of one
 * after the other).  Jobs are queued at submit, admitted in arrival order
 * while their device footprint fits the server's HBM budget (and at most
 * max_jobs are admitted), and their work is interleaved on the GPU in epochs
 * of about epoch_target_ms: work of jobs that arrive while others run
 * overlaps with theirs.  A job's result is the same, bit for bit, whether it
 * ran alone or in a mix.
 */
typedef struct ccm_server ccm_server;

typedef struct {
  uint64_t hbm_budget_bytes;  /* device arena for job data; 0 = default
                                 (a quarter of free memory, at most 32 GiB) */
  int32_t max_jobs;           /* admitted at once; <= 0 = 64 */
  double epoch_target_ms;     /* device time per epoch; <= 0 = 20 ms */
} ccm_server_cfg;

/* One job: as ccm() (both directions, one E and tau).  Every array is
   copied at submit; flags in opts are ignored. */
typedef struct {
  const double *X, *Y;
  int64_t N;
  int32_t E, tau;
  const int64_t *L;
  int32_t nL;
  int32_t r;
  uint64_t seed;
  ccm_opts opts;
} ccm_job;

/* Seconds since the server was created; work counts of the job; the
   device bytes it held while admitted (its footprint against the budget). */
typedef struct {
  double t_submit, t_admit, t_done;
  uint64_t pairs, predictions, realizations;
  uint64_t device_bytes;
} ccm_job_stats;

/* Start a server on the context's device (its own stream and thread). */
ccm_status ccm_server_create(ccm_ctx *ctx, const ccm_server_cfg *cfg,
                             ccm_server **out);
/* Queue a job; never waits for the GPU.  CCM_E_INVAL for a malformed job
   or one whose opts.flags ask for CCM_FLAG_NESTED or CCM_FLAG_SHARED_E (they
   change the draws and are not served), CCM_E_NOMEM if its footprint (tables
   included) exceeds the whole budget.  CCM_FLAG_TABLE is honoured; the other
   flags choose an execution form, which the server picks itself, and are
   ignored. */
ccm_status ccm_submit(ccm_server *srv, const ccm_job *job, uint64_t *ticket);
/* Wait until the job is finished (timeout_ns < 0: no limit).
   CCM_E_TIMEOUT if it is not finished in time, CCM_E_NOTFOUND for an unknown
   or cancelled ticket, the job's error status if it failed.  A job cancelled
   while running counts as finished once its in-flight device work is done. */
ccm_status ccm_wait(ccm_server *srv, uint64_t ticket, int64_t timeout_ns);
/* Copy a finished job's rho (host double[nL][r] each, nullable) and stats,
   and release the ticket.  CCM_E_BUSY while the job is still running, also
   when it was cancelled and its in-flight device work is not done yet (the
   ticket is then kept); CCM_E_NOTFOUND, releasing the ticket, for a job
   cancelled and finished. */
ccm_status ccm_result(ccm_server *srv, uint64_t ticket, double *rho_X_from_MY,
                      double *rho_Y_from_MX, ccm_job_stats *stats);
/* Cancel a queued or running job (its remaining work is skipped; work
   already on the device completes before the job is released). */
ccm_status ccm_cancel(ccm_server *srv, uint64_t ticket);
/* Cancel everything outstanding, wait for the device, release the server. */
void ccm_server_destroy(ccm_server *srv);

/*
 * Test hook: the library subsample the sampler draws for realization
 * r_index of (E, tau, L_eff) under seed, over N_e embedded points.
 *   idx_out     host int32[L_eff], ascending embedded-point indices
 */
ccm_status ccm_library(ccm_ctx *ctx, int64_t N_e, int32_t E, int32_t tau,
                       int64_t L_eff, int32_t r_index, uint64_t seed,
                       int32_t *idx_out);

/*
 * Test hook: the first n_out points of the nested ordering that
 * CCM_FLAG_NESTED draws for realization r_index of (E, tau) under seed, over
 * N_e embedded points (the library of size L_eff is its first L_eff points).
 *   idx_out     host int32[n_out], in drawing order; 1 <= n_out <= N_e
 */
ccm_status ccm_nested_library(ccm_ctx *ctx, int64_t N_e, int32_t E, int32_t tau,
                              int32_t r_index, uint64_t seed, int64_t n_out,
                              int32_t *idx_out);

/*
 * Test hook: one realization over a caller-given library (Section 3.2 and
 * 2.1), with every per-query result exported.
 *   lib_series  host double[N]: series whose manifold is searched
 *   target      host double[N]: series that is predicted
 *   lib_idx     host int32[L_eff]: strictly ascending embedded indices
 *   nbr         host int32[Nq][E+1] (nullable): neighbour indices, nearest
 *               first; Nq = N_e, or L_eff with query_set = 1
 *   d2          host float[Nq][E+1] (nullable): their squared distances
 *   pred        host double[Nq] (nullable): predictions
 *   rho         host double (nullable): the skill
 * With CCM_FLAG_TABLE in opts->flags the realization walks a distance
 * indexing table over the embedding whatever its size (the walk, and its
 * fallback to the scan when a row runs short, give the same results).
 */
ccm_status ccm_neighbors(ccm_ctx *ctx, const double *lib_series,
                         const double *target, int64_t N, int32_t E,
                         int32_t tau, const int32_t *lib_idx, int64_t L_eff,
                         const ccm_opts *opts, int32_t *nbr, float *d2,
                         double *pred, double *rho);

/* Kernel timing of the cross-map kernels (HIP events on the launch stream).
   While enabled, batched calls issue their launches directly (no graph: the
   runtime cannot time events recorded by graph nodes). */
typedef struct {
  double kernel_ms;      /* summed duration of cross-map kernel launches */
  int64_t launches;      /* cross-map kernel launches timed */
  double pairs;          /* (query, candidate) distance evaluations */
  double flops;          /* 3E-1 binary32 flops per pair, summed */
  double predictions;    /* cross-map predictions made */
  double realizations;   /* rho values produced */
  double table_realizations; /* of which walked a distance indexing table */
  double waves;          /* waves of realizations run (ccm_set_wave_limit) */
} ccm_profile;

ccm_status ccm_profile_enable(ccm_ctx *ctx, int on);
/* Wait for the timed launches, fill *out, and zero the counters if reset. */
ccm_status ccm_profile_read(ccm_ctx *ctx, ccm_profile *out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* CCM_H */
