/*
 * librtdetmcd -- RT-DetMCD (arXiv 1910.05615) on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Unless stated otherwise every data
 * pointer is a DEVICE pointer on the handle's device, owned by the caller, and
 * every call is asynchronous on the handle's stream.  Matrices are row-major.
 * Status codes are returned synchronously for argument errors; data-dependent
 * outcomes are reported in device-side status arrays.  No C++ exception
 * crosses this boundary.  One handle must not be used from two host threads at
 * once.
 *
 * Method references:
 *   Sec. 2.1   raw MCD (eq. mcdraw), statistical distance (eq. statdist),
 *              C-step (eq. cstep1 .. cstep4b), reweighting and flagging
 *   Sec. 3.1   univariate reweighted MCD standardisation
 *   Sec. 3.2   wrapping (eq. wrapping) and GSSCM (eq. LR) initial estimators
 *   Sec. 3.3   refinement of the initial estimators
 *   Sec. 3.4   Cholesky distances and condition monitor (eq. choleskymonitor)
 *   Sec. 3.5   update-based C-step (eq. propcstep1, muUpdate, propcstep2)
 *   Sec. 4     blocks, entrywise median, KL deviation (eq. KL), pooling
 *              (eq. covpool1, covpool2), distributed reweighting, flags
 *   Sec. 5     block-count rule (eq. partitionsize)
 */
#ifndef RTDETMCD_H
#define RTDETMCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
typedef int32_t rtdetmcd_status;
#define RTDETMCD_OK            0
#define RTDETMCD_EINVAL       -1   /* bad argument (sizes, h out of (p, m), null) */
#define RTDETMCD_ENOMEM       -2   /* device allocation of the workspace failed */
#define RTDETMCD_EDEVICE      -3   /* HIP runtime error (message in last_error) */
#define RTDETMCD_ESINGULAR    -4   /* no block produced a valid fit */
#define RTDETMCD_ENONFINITE   -5   /* X holds NaN or Inf (fits: that dataset; its outputs are
                                      not meaningful) */
#define RTDETMCD_EUNSUPPORTED -6   /* p > RTDETMCD_MAX_P, too many blocks */

#define RTDETMCD_MAX_P 64

/* data types of X */
#define RTDETMCD_F32 0
#define RTDETMCD_F64 1

/* Per-start / per-block status values written to device arrays.  A block's
 * status is that of its chosen start; RTDETMCD_BLOCK_INVALID marks a block
 * whose two starts were both dropped (excluded from aggregation, Sec. 4 step 4). */
#define RTDETMCD_ST_CONVERGED   0  /* h-subset repeated (Sec. 2.2 step 4) */
#define RTDETMCD_ST_NOTCONV     1  /* max_csteps reached; fit still usable */
#define RTDETMCD_ST_ILLCOND     2  /* next C-step refused by the condition monitor (Sec. 3.4) */
#define RTDETMCD_ST_DROP_REFINE 3  /* start dropped in refinement (Sec. 3.3 step 2) */
#define RTDETMCD_ST_DROP_FIRST  4  /* start refused before its first C-step */
#define RTDETMCD_ST_SINGULAR    5  /* a subset covariance was not positive definite */
#define RTDETMCD_BLOCK_INVALID  3

/* option values */
#define RTDETMCD_STD_UNIMCD 0   /* univariate reweighted MCD (Sec. 3.1) */
#define RTDETMCD_STD_MEDMAD 1   /* median and 1.4826 MAD */
#define RTDETMCD_CSTEP_FULL   0 /* recompute the subset mean / covariance (eq. cstep4a, cstep4b) */
#define RTDETMCD_CSTEP_UPDATE 1 /* update from the swapped rows only (Sec. 3.5) */
#define RTDETMCD_CSTEP_AUTO   2 /* update, with a full recompute when many rows swap */
#define RTDETMCD_CSTEP_SMW    3 /* AUTO, and a step whose subset changed by one row out and one
                                  in updates the inverse of the sscp matrix by the
                                  Sherman-Morrison-Woodbury identity and its determinant by
                                  the ratio Delta_i (Sec. 3.5, eq. woodbury, scaleddetUpdate);
                                  the next step's distances use that inverse */
#define RTDETMCD_DIST_CHOLESKY 0 /* distances by forward substitution with the Cholesky
                                   factor (Sec. 3.4) */
#define RTDETMCD_DIST_INVERSE  1 /* distances (x-mu)^T Sigma^{-1} (x-mu) with the explicit
                                   inverse, every distance of the fit (the I versus ID rows
                                   of Table 1, Sec. 5) */
#define RTDETMCD_START_WARM    2 /* block_start of a block fitted from a warm start */
#define RTDETMCD_POOL_PRINTED 0 /* Sec. 4 step 7 formulas with block counts m */
#define RTDETMCD_POOL_UNION   1 /* the text of Sec. 4 step 7: classical mean and
                                  covariance of the union of the kept blocks'
                                  h-subsets, times c(h/m) */
#define RTDETMCD_LAUNCH_BATCHED 0 /* every block and start in the same launches */
#define RTDETMCD_LAUNCH_PLAIN   1 /* one block, one start at a time, host-driven */

typedef struct rtdetmcd_opts {
  int32_t struct_size;      /* sizeof(rtdetmcd_opts) */
  double  alpha;            /* h = floor(alpha m) when h_sub == 0 (default 0.75) */
  int32_t standardize;      /* RTDETMCD_STD_* (default UNIMCD) */
  int32_t cstep_mode;       /* RTDETMCD_CSTEP_* (default AUTO) */
  int32_t max_csteps;       /* default 100 */
  double  kappa_max;        /* condition bound, default 1000 (Sec. 3.3, 3.4) */
  double  cutoff_q;         /* chi-square quantile of the cutoff, default 0.975 */
  int32_t pool_mode;        /* RTDETMCD_POOL_* (default PRINTED) */
  int32_t rew_consistency;  /* 1: multiply the reweighted scatter by c(cutoff_q) (default 0) */
  int32_t omega;            /* block-count rule bound (default 4096) */
  int32_t launch;           /* RTDETMCD_LAUNCH_* (default BATCHED) */
  int32_t graph;            /* 1: replay the C-step rounds from a captured hipGraph */
  int32_t rounds_per_sync;  /* C-steps enqueued between host checks of convergence (default 4) */
  int32_t distance;         /* RTDETMCD_DIST_* (default CHOLESKY) */
  int32_t tune;             /* 1: autotune the batched C-step loop (default 0): on the first
                             * fit of a shape (p bucket, item count, rows, longest block,
                             * input type) the library times the distance pass of the
                             * first C-step under each candidate tiling (rows per tile
                             * 256..4096) and keeps the fastest; later fits of that shape take
                             * the kept tiling, and their first convergence check comes
                             * after as many C-steps as the previous fit took (at least
                             * rounds_per_sync).  Results do not depend on it. */
} rtdetmcd_opts;

/* Output buffers of a fit.  Every field is a caller-allocated device buffer or
 * NULL ("do not produce").  Sizes use q, m, h from rtdetmcd_plan.  Location and
 * scatter are in the units of X. */
typedef struct rtdetmcd_out {
  double*  mu;            /* [p]   reweighted location (Sec. 4 step 9) */
  double*  sigma;         /* [p*p] reweighted scatter */
  double*  mu_raw;        /* [p]   aggregated raw location (Sec. 4 step 7) */
  double*  sigma_raw;     /* [p*p] aggregated raw scatter */
  double*  logdet;        /* [2]   log det of sigma_raw, sigma */
  double*  dist;          /* [n]   final robust distances (Sec. 4 step 10) */
  uint8_t* outlier;       /* [n]   1 iff squared distance > chi2_{p,cutoff_q} */
  int32_t* hsubset;       /* [q*h] chosen h-subset of each block, ascending row indices of X */
  int32_t* block_status;  /* [q]   RTDETMCD_ST_* of the chosen start, or BLOCK_INVALID */
  int32_t* block_start;   /* [q]   0 = wrapping start, 1 = GSSCM start, RTDETMCD_START_WARM
                           *       for a warm start, -1 none */
  int32_t* block_iters;   /* [q]   C-steps taken by the chosen start */
  double*  loc;           /* [p]   standardisation location (Sec. 3.1) */
  double*  scale;         /* [p]   standardisation scale */
  int64_t* n_w;           /* [1]   rows kept by the reweighting */
  uint8_t* rew_mask;      /* [n]   1 for the rows kept by the reweighting (Sec. 4 step 8:
                           *       fitted rows whose squared distance under the raw fit
                           *       does not exceed chi2_{p,cutoff_q}), 0 otherwise */
  /* Diagnostics of rtdetmcd_fit / rtdetmcd_fit_batched (other calls ignore
   * them), computed only when non-NULL: */
  double*  ldtrace;       /* [q*max_csteps] per block, log det of the chosen start's scatter
                           *       (standardised units) at each evaluated C-step, in order:
                           *       non-increasing for full steps (Sec. 2.1, the C-step
                           *       theorem); NaN from block_iters on */
  double*  hmargin;       /* [q]   per block, d2_(h+1) - d2_(h) of the chosen start's last
                           *       evaluated squared distances (Sec. 2.1 eq. cstep3): the gap
                           *       at the h-subset threshold, 0 for a tie; NaN for an invalid
                           *       block */
  double*  cmargin;       /* [1]   smallest |dist^2 - chi2_{p,cutoff_q}| over the final
                           *       distances (Sec. 4 step 10): the margin of the outlier
                           *       flags; needs `dist`, NaN without it */
} rtdetmcd_out;

typedef struct rtdetmcd_ctx* rtdetmcd_handle;

/* Create a handle on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The handle owns a device workspace that grows on
 * demand and is freed by rtdetmcd_destroy.  Columns longer than one LDS
 * segment are sorted by buckets (a sample sort) or by global radix passes,
 * both ranking with LDS atomics and checked; a fit whose check fails, or
 * whose bucket overflows, is run again with the full-width radix sort and
 * ballot ranking only (counted by rtdetmcd_sort_reruns).
 * RTDETMCD_SAFE_SORT=1 in the environment at creation selects that sort
 * from the start. */
rtdetmcd_status rtdetmcd_create(rtdetmcd_handle* out, int32_t device, void* hip_stream);
rtdetmcd_status rtdetmcd_destroy(rtdetmcd_handle h);
rtdetmcd_status rtdetmcd_set_stream(rtdetmcd_handle h, void* hip_stream);
/* Message of the last error on this handle (valid until the next call). */
const char* rtdetmcd_last_error(rtdetmcd_handle h);

/* The autotuned plans a handle holds (opts.tune), most recent last: up to
 * `cap` rows of 4 int64 (p bucket, rows per distance tile, items per
 * distance tile (1), C-steps of the last fit) into `out` (host memory, may
 * be NULL when cap = 0).  *count
 * receives the number of plans held.  Errors: RTDETMCD_EINVAL for a null
 * handle or count. */
rtdetmcd_status rtdetmcd_tuned_plans(rtdetmcd_handle h, int64_t* out, int32_t cap,
                                     int32_t* count);
/* Paper defaults (Sec. 2.1, 3.3, 3.4, 5). */
void rtdetmcd_default_opts(rtdetmcd_opts* o);

/* Block count q, block length m = floor(n/q) and subset size h of a fit
 * (host-only).  n_chunks == 0 applies q = max(floor(n/(p omega)), 1)
 * (eq. partitionsize); h_sub == 0 applies h = floor(alpha m) clamped into
 * [(m+p+1)/2, m-1] (Sec. 2.1).  EINVAL unless p < h < m and n > 2p. */
rtdetmcd_status rtdetmcd_plan(int64_t n, int32_t p, int64_t h_sub, int32_t n_chunks,
                              const rtdetmcd_opts* o, int32_t* q, int64_t* m, int64_t* h);

/* Full RT-DetMCD fit of X (n x p, row stride ld elements, dtype F32 or F64)
 * (Sec. 4 steps 1-10; q = 1 is the serial version).  Blocks are the
 * contiguous row ranges [l m, (l+1) m); the n - q m remainder rows are not
 * fitted but are scored and flagged.  Synchronises the stream once at the end
 * to read the validity of the blocks; returns ESINGULAR if none is valid. */
rtdetmcd_status rtdetmcd_fit(rtdetmcd_handle h, const void* X, int32_t dtype, int64_t n,
                             int32_t p, int64_t ld, int64_t h_sub, int32_t n_chunks,
                             const rtdetmcd_opts* o, const rtdetmcd_out* out);

/* Many independent datasets fitted in the same launches.  `sets` is a HOST
 * array of n_datasets descriptors; each descriptor's X and out are device
 * buffers as for rtdetmcd_fit.  status[i] (host) receives each dataset's code.
 *
 * perm (device, int32 [n], or NULL): the random partition of Sec. 4 — block l
 * is rows perm[l m], ..., perm[(l+1) m - 1] of X, and rows perm[q m .. n) are
 * the unfitted remainder (still scored and flagged).  The caller draws the
 * permutation (the library draws no random numbers); NULL means contiguous
 * blocks [l m, (l+1) m).  The library copies the q m fitted rows into its
 * workspace in block order.  A perm that is not a permutation of 0 .. n-1
 * (an entry out of range or repeated) gives that dataset RTDETMCD_EINVAL;
 * out-of-range entries are never used as row indices.  With a perm, hsubset
 * lists each block's subset as rows of X in order of their position within
 * the block (ascending only for contiguous blocks), and rew_mask and the
 * final distances stay in the row order of X.
 *
 * warm_mu (device, float64 [p]) and warm_sigma (device, float64 [p*p],
 * row-major), both non-NULL: the warm start of the last paragraph of Sec. 4.
 * A previous fit's reweighted location and scatter (units of X) become the
 * one start of every block's C-steps (Sec. 4 step 3); the initial estimators
 * and their refinement (steps 1-2) are not computed for that dataset.  The
 * standardisation of the new data and steps 4-10 run as usual.  A warm start
 * that is not positive definite or too ill-conditioned leaves the blocks
 * invalid (RTDETMCD_ESINGULAR).  Both NULL: the usual two starts. */
typedef struct rtdetmcd_dataset {
  const void* X; int32_t dtype; int64_t n; int32_t p; int64_t ld;
  int64_t h_sub; int32_t n_chunks; rtdetmcd_out out;
  const int32_t* perm;
  const double* warm_mu;
  const double* warm_sigma;
} rtdetmcd_dataset;
rtdetmcd_status rtdetmcd_fit_batched(rtdetmcd_handle h, int32_t n_datasets,
                                     const rtdetmcd_dataset* sets, const rtdetmcd_opts* o,
                                     rtdetmcd_status* status);

/* ---- host-only distribution helpers (no device work) --------------------- */

/* Quantile and CDF of the chi-square distribution with df degrees of freedom
 * (regularised incomplete gamma by its power series / continued fraction;
 * quantile by bisection), and the consistency factor
 * c(alpha) = alpha / F_{chi2_{p+2}}(chi2_{p,alpha}) of the raw MCD scatter
 * (Sec. 2.1, eq. mcdraw; the factor the paper cites without printing). */
double rtdetmcd_chi2_quantile(double q, int32_t df);
double rtdetmcd_chi2_cdf(double x, int32_t df);
double rtdetmcd_consistency(double alpha, int32_t p);

/* ---- low-level steps (parity tests and composition) ---------------------- */

/* Squared statistical distances d2[i] = ||L^{-1}(x_i - mu)||^2 of the n rows
 * of X, with L the lower Cholesky factor of Sigma (eq. statdist via Sec. 3.4).
 * mu [p] and L [p*p, lower triangle read] are device float64.  n = 0 returns
 * RTDETMCD_OK without reading or writing anything (pointers may be NULL). */
rtdetmcd_status rtdetmcd_distances(rtdetmcd_handle h, const void* X, int32_t dtype, int64_t n,
                                   int32_t p, int64_t ld, const double* mu, const double* L,
                                   double* d2);

/* Robust distances and outlier flags of n rows against a stored fit: the
 * last step of Sec. 4 (step 10), used on its own to score new data against a
 * trained fit (Sec. 6).  mu [p] and Linv [p*p] are device float64; Linv is the
 * inverse of the lower Cholesky factor of Sigma, row-major (lower triangle
 * read), so that d2_i = ||Linv (x_i - mu)||^2.  dist [n] (float64, nullable)
 * receives sqrt(d2_i); outlier [n] (nullable) receives d2_i > cut, with
 * cut <= 0 meaning chi2_{p,0.975}.  One kernel launch; n = 0 returns
 * RTDETMCD_OK without reading or writing anything (pointers may be NULL). */
rtdetmcd_status rtdetmcd_score(rtdetmcd_handle h, const void* X, int32_t dtype, int64_t n,
                               int32_t p, int64_t ld, const double* mu, const double* Linv,
                               double cut, double* dist, uint8_t* outlier);

/* Indices of the h_sub smallest d2 values, ties broken by the smaller index
 * (C-step steps 2-3 of Sec. 2.1).  idx [h_sub] receives them ascending; mask
 * [m] (nullable) receives 1 for selected rows and 0 otherwise.  Exact: the
 * comparison is on the float64 bit patterns. */
rtdetmcd_status rtdetmcd_select(rtdetmcd_handle h, const double* d2, int64_t m, int64_t h_sub,
                                int32_t* idx, uint8_t* mask);

/* C-steps on one block X (m x p) from the start (mu0, sigma0) until the
 * h-subset repeats (Sec. 2.1, 3.4, 3.5).  kappa_scale [p] (nullable) gives the
 * column scales by which sigma is divided before the condition check, so that
 * the check acts in standardised units.  Outputs (device): mu [p], sigma [p*p]
 * (subset covariance, divisor h-1), hsubset [h_sub] ascending, status [1],
 * iters [1], logdet [1]. */
rtdetmcd_status rtdetmcd_cstep(rtdetmcd_handle h, const void* X, int32_t dtype, int64_t m,
                               int32_t p, int64_t ld, int64_t h_sub, const double* mu0,
                               const double* sigma0, const double* kappa_scale,
                               const rtdetmcd_opts* o, double* mu, double* sigma,
                               int32_t* hsubset, int32_t* status, int32_t* iters,
                               double* logdet);

/* The C-steps of rtdetmcd_cstep (same arguments, same kernels, same results)
 * for callers that cannot allocate memory: code that runs while a stream is
 * being captured, tight serving loops, harnesses that forbid allocation.  It
 * calls no hipMalloc / hipFree and no allocating library routine; every device
 * buffer beyond the caller's inputs and outputs comes from one fixed array of
 * 8 MiB that the library holds on each device it runs on until the process
 * ends.  Limit: m <= 131072 rows (p <= RTDETMCD_MAX_P); a larger m returns
 * RTDETMCD_EINVAL with a message.  opts->graph is ignored (capturing a graph
 * allocates).  All calls on one device share that array and each call leaves
 * its state there: calls that overlap on one device (two host threads, or two
 * streams whose work overlaps) race and give wrong results.  Like
 * rtdetmcd_cstep it synchronises the stream between C-steps to test for
 * convergence. */
rtdetmcd_status rtdetmcd_cstep_noalloc(rtdetmcd_handle h, const void* X, int32_t dtype,
                                       int64_t m, int32_t p, int64_t ld, int64_t h_sub,
                                       const double* mu0, const double* sigma0,
                                       const double* kappa_scale, const rtdetmcd_opts* o,
                                       double* mu, double* sigma, int32_t* hsubset,
                                       int32_t* status, int32_t* iters, double* logdet);

/* ---- kernel timing -------------------------------------------------------- */

/* Kernel classes timed by rtdetmcd_profile_read. */
#define RTDETMCD_PROF_SEGSORT    0 /* LDS segment sort + univariate MCD / order statistics
                                      (standardisation of short columns, GSSCM norms, the
                                      refinement's score columns); bytes: keys read + results */
#define RTDETMCD_PROF_CSTEP_DIST 1 /* distance pass of the first C-step (every start active);
                                      bytes: rows read + float64 d2 written; flops: p(p+1)+3p
                                      per row and start */
#define RTDETMCD_PROF_SELECT     2 /* h-subset selection of the first C-step; bytes: d2 read,
                                      mask written */
#define RTDETMCD_PROF_SSCP       3 /* subset sums of the first (full) C-step on the matrix
                                      cores; bytes: rows and mask read; flops useful: h (p+1)
                                      (p+2) per start (lower triangle with sums and count),
                                      executed: the 16 x 16 x 4 blocks over every row */
#define RTDETMCD_PROF_FINALIZE   4 /* Cholesky / inverse / condition step of the first C-step */
#define RTDETMCD_PROF_FINAL_DIST 5 /* final distances and flags of every row (Sec. 4 step 10);
                                      bytes: rows read, distance, flag and weight written,
                                      the reweighting distances read */
#define RTDETMCD_PROF_FIT        6 /* a whole fit, first launch to last */
#define RTDETMCD_PROF_DISTANCES  7 /* the distance kernel of rtdetmcd_distances / the scoring
                                      kernel of rtdetmcd_score; bytes: rows read, results
                                      written; flops: p(p+1)+3p per row */
#define RTDETMCD_PROF_KINDS      8

/* Kernel timing of the fits that follow on this handle: enable = 1 clears the
 * records and starts recording a HIP event on the handle's stream before and
 * after each launch of the classes above (eager launches only: the C-step
 * rounds replayed from a graph are not timed, the first C-step always runs
 * eagerly while timing is on); 0 stops.  Host-side bookkeeping only. */
rtdetmcd_status rtdetmcd_profile(rtdetmcd_handle h, int32_t enable);
/* Totals over the recorded launches of one class (synchronises the stream):
 * milliseconds between the events, launches, algorithmic bytes and flops
 * (useful, and executed by the matrix cores where that differs).  Every
 * pointer may be NULL. */
rtdetmcd_status rtdetmcd_profile_read(rtdetmcd_handle h, int32_t kind, double* ms,
                                      int64_t* launches, double* bytes, double* flops_useful,
                                      double* flops_exec);

/* Number of fits on this handle that were run a second time on the
 * full-width, ballot-ranked sort because a long-column sort's check failed or
 * a bucket of the sample sort overflowed (see rtdetmcd_create).
 * Such a fit takes about twice its usual time; its results are those of the
 * ballot-ranked run.  Host-only; -1 for a null handle. */
int64_t rtdetmcd_sort_reruns(rtdetmcd_handle h);

/* ---- adjoint -------------------------------------------------------------- */

/* Gradient with respect to X of <g_dist, dist> + <g_mu, mu> + <g_sigma, sigma>
 * for a finished fit, with the reweighting set held fixed.  The fit ends with
 * mu = mean and sigma = c_rew * covariance (divisor n_w - 1) of the rows of W,
 * and dist_i = ||sigma^{-1/2}(x_i - mu)|| for every row (Sec. 4 steps 9-10,
 * eq. statdist).  W, like the h-subsets, is constant away from ties at the
 * cutoff, so this is the derivative of the fit wherever it exists.
 * Inputs (device): X and its shape as given to the fit; mu [p], sigma [p*p],
 * dist [n], rew_mask [n] and n_w [1] from the fit's rtdetmcd_out; c_rew (host)
 * the scatter factor of the fit (1, or the consistency factor when
 * rew_consistency was set).  Cotangents (device float64, each nullable = 0):
 * g_dist [n], g_mu [p], g_sigma [p*p] (row-major; its symmetric part acts).
 * Output: g_X [n*p] float64, row-major with row stride p.  Rows with
 * dist_i = 0 receive no term from their own distance.  Asynchronous. */
rtdetmcd_status rtdetmcd_backward(rtdetmcd_handle h, const void* X, int32_t dtype, int64_t n,
                                  int32_t p, int64_t ld, const double* mu, const double* sigma,
                                  const double* dist, const uint8_t* rew_mask,
                                  const int64_t* n_w, double c_rew, const double* g_dist,
                                  const double* g_mu, const double* g_sigma, double* g_X);

#ifdef __cplusplus
}
#endif
#endif /* RTDETMCD_H */
