/*
 * enkfmc.h -- C ABI of the MI355X EnKF-MC hot path.
 *
 * The library computes, for a background ensemble X_b (n x N), the analysis
 * ensemble of the ensemble Kalman filter based on the modified Cholesky
 * decomposition (arXiv 1606.00807):
 *
 *   - Section 3 / Alg. 2: the grid is split into Delta = sdx*sdy sub-domains,
 *     each extended by a halo of r_h grid points;
 *   - eq. (1), eq. (8), Alg. 3 first step: in every sub-domain each component's
 *     ensemble anomalies are regressed on its predecessors inside its local box
 *     of radius r (Section 2.3, text after eq. 9), giving B^-1 ~ T^T D^-1 T;
 *   - eq. (11) per sub-domain (eq. 14, Alg. 3): the local analysis increment
 *     solves (T^T D^-1 T + H^T R^-1 H) dX = H^T R^-1 (Y^s - H X_b);
 *   - Alg. 2 merge step: interior rows are written back to the global grid.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Global ordering: variable-major, then level, then latitude, then
 *    longitude (longitude fastest).  Component g = off_v + (lev*ny + lat)*nx + lon.
 *  - Matrices are row-major with the N members of one component contiguous:
 *    X_b and X_a are (n, N), Y^s is (m, N).
 *  - H is a selection: obs_idx[o] is the component observed by observation o
 *    (strictly increasing, inside [0, n)).  R is diagonal: r_diag[o] > 0.
 *  - Sub-domain k = ky*sdx + kx.  Its local rows are ordered variable, level,
 *    local latitude, local longitude over its extended box.  Predecessors are
 *    same-variable rows earlier in that local order with |dlev| <= r_v,
 *    |dlat| <= r_h, |dlon| <= r_h.  With sdx == 1 and a periodic grid there is
 *    no longitude halo and longitude distance is periodic.
 *  - Arguments named "dev" point to device memory, "host" to host memory.
 *  - A stream argument is a hipStream_t passed as void* (NULL: null stream).
 *    Every device call is ordered on that stream and ends with one small
 *    device-to-host read of a status word, so it returns only after its work
 *    has finished -- unless the plan is in asynchronous mode
 *    (enkfmc_set_async), where calls only enqueue their kernels.
 *  - No entry point throws.  On failure a negative status is returned and
 *    enkfmc_last_error() describes it (per calling thread).
 *  - A plan is not re-entrant: calls on one plan must not overlap.  Distinct
 *    plans are independent.
 */
#ifndef ENKFMC_H
#define ENKFMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ENKFMC_OK = 0,
  ENKFMC_EINVAL = -1,       /* bad argument, geometry or observation list          */
  ENKFMC_ENOTSPD = -2,      /* a regression or innovation matrix is not SPD        */
  ENKFMC_ENONPOS_D = -3,    /* a residual variance D_ii is not positive            */
  ENKFMC_ENOCONV = -4,      /* iterative solve did not converge within its limit   */
  ENKFMC_EHIP = -5,         /* HIP runtime error                                   */
  ENKFMC_ENOMEM = -6,       /* workspace too small or host allocation failed       */
  ENKFMC_ESTATE = -7,       /* call out of order (e.g. analyze before fit)         */
  ENKFMC_EUNSUPPORTED = -8  /* sizes beyond what the kernels were built for        */
} enkfmc_status;

typedef enum { ENKFMC_F32 = 0, ENKFMC_F64 = 1 } enkfmc_dtype;

/* How enkfmc_fit computes the regressions (same result within rounding). */
typedef enum {
  ENKFMC_FIT_PLAIN = 0,   /* one workgroup per regression, FP64 vector arithmetic */
  ENKFMC_FIT_BATCHED = 1, /* one wavefront per regression, FP64 MFMA Gram, register Cholesky */
  ENKFMC_FIT_SVD = 2      /* one workgroup per regression: SVD of its design matrix by
                             one-sided Jacobi (the route of Section 5), FP64 */
} enkfmc_fit_mode;

/* How enkfmc_analyze solves the local systems (same result within rounding). */
typedef enum {
  ENKFMC_SOLVE_DUAL = 0,  /* direct: dual form eqs. (12)-(13) per variable block  */
  ENKFMC_SOLVE_PCG = 1    /* iterative: conjugate gradients on the primal eq. (11)
                             per (block, member), preconditioned by B^ = T^-1 D T^-T
                             (eq. 8), FP64 with residual refinement */
} enkfmc_solver;

typedef struct {
  int32_t nx, ny;          /* horizontal grid; longitude fastest                     */
  int32_t nvar;            /* number of variables                                    */
  const int32_t *nlev;     /* host [nvar]: levels of each variable (>= 1)            */
  int32_t periodic_x;      /* 1: longitude wraps                                     */
  int32_t sdx, sdy;        /* sub-domain tiles in longitude and latitude             */
  int32_t r_h, r_v;        /* radius of influence (horizontal, vertical)            */
} enkfmc_geometry;

typedef struct enkfmc_plan enkfmc_plan;

typedef struct {
  int64_t n;               /* state size                                             */
  int64_t N;               /* ensemble size                                          */
  int64_t m;               /* observations                                           */
  int64_t n_subdomains;    /* Delta                                                  */
  int64_t n_blocks;        /* (sub-domain, variable) blocks                          */
  int64_t n_fit;           /* local rows over all sub-domains (regressions)          */
  int64_t nnz;             /* strictly-lower entries of T over all sub-domains       */
  int64_t m_local;         /* local observations over all sub-domains                */
  int32_t max_p;           /* largest predecessor count                              */
  int32_t max_block_rows;  /* largest block                                          */
  int32_t max_block_obs;   /* most observations in one block                         */
  int32_t reserved;
  size_t workspace_bytes;  /* device workspace enkfmc_plan_set_workspace needs       */
  int64_t fit_rows_wave;   /* rows ENKFMC_FIT_BATCHED fits with one-wavefront kernels */
  int64_t fit_rows_plain;  /* rows ENKFMC_FIT_BATCHED hands to the plain kernel       */
  int64_t n_row_tiles;     /* 16-row tiles of T over all blocks                      */
  int64_t n_tiles;         /* stored off-diagonal 16x16 tiles of T                   */
  int64_t f_entries;       /* entries of the dual form's F = T^-T H^T, all blocks     */
  int64_t s_entries;       /* entries of its S = R + F^T D F, all blocks              */
  size_t factor_cache_bytes; /* memory enkfmc_plan_set_factor_cache needs      */
  /* Row-tile distances R - C of the stored tiles T_RC (C < R) of T, which
   * decide the form of the triangular sweeps: every distance 1..near_d
   * occurs (at most 8); far_lo is the smallest distance beyond near_d (0 if
   * none), max_tile_distance the largest, and far_ring the widest range of
   * distances beyond near_d within one block.                              */
  int32_t near_d, far_lo, max_tile_distance, far_ring;
} enkfmc_plan_info;

/* Build the decomposition of Section 3 (host only, no device work).
 * g: geometry; N >= 2 members; obs_idx (host, m entries, strictly increasing,
 * inside [0, n)).  On success *out owns the plan (enkfmc_plan_destroy). */
enkfmc_status enkfmc_plan_create(enkfmc_plan **out, const enkfmc_geometry *g, int32_t N,
                                 const int32_t *obs_idx, int32_t m);

enkfmc_status enkfmc_plan_get_info(const enkfmc_plan *p, enkfmc_plan_info *info);

/* Hand the plan caller-owned device memory of at least info.workspace_bytes
 * (256-byte aligned) and upload the index maps into it.  The plan keeps the
 * pointer; the caller keeps the memory alive until the plan is destroyed or
 * given another workspace. */
enkfmc_status enkfmc_plan_set_workspace(enkfmc_plan *p, void *dev, size_t bytes, void *stream);

/* Optional cache of the regressions' Cholesky factors (eq. 1, each solved as
 * a p x p system, or as its N x N kernel system when p >= N) for the reverse
 * pass.  dev: caller-owned device memory of at least info.factor_cache_bytes
 * (256-byte aligned; T(T + 1)/2 x 2 KiB per regression of the one-wavefront
 * kernels with predecessors, T = ceil(min(p, N)/16): 30 KiB at p or N = 80),
 * or NULL to drop the cache.  While set, every ENKFMC_FIT_BATCHED fit writes
 * each such row's factored tiles there, and enkfmc_analyze_backward after
 * that fit reads them instead of recomputing the row's Gram and Cholesky.
 * The result differs from the recomputing reverse pass only by rounding.
 * The plan keeps the pointer; setting or dropping the cache invalidates what
 * it holds until the next fit.  Errors: EINVAL (NULL plan, misaligned),
 * ENOMEM (too small). */
enkfmc_status enkfmc_plan_set_factor_cache(enkfmc_plan *p, void *dev, size_t bytes);

/* Fit B^-1 = T^T D^-1 T in every sub-domain (eq. 1, eq. 8; Alg. 3 first step).
 * Xb: dev (n x N), element type dtype, row stride ld >= N elements.
 * ridge >= 0 is added to the (N-1)-normalised Gram of every regression; with
 * ridge == 0 a regression with N - 1 or more predecessors is ENOTSPD.
 * mode: enkfmc_fit_mode.  ENKFMC_FIT_BATCHED fits every regression with a
 * one-wavefront kernel when N <= 128 and it has at most 192 predecessors;
 * the other regressions (all of them when (n + 2) * ldu reaches 2^31, ldu =
 * N rounded up to a multiple of 16) go to the plain kernel, which the
 * counts fit_rows_wave / fit_rows_plain of enkfmc_plan_info report.
 * T and D stay in the workspace.
 * ENKFMC_FIT_SVD computes beta = V diag(sigma/(sigma^2 + mu)) W^T u from the
 * SVD U_P^T = W diag(sigma) V^T (mu = ridge (N - 1)), the same coefficients
 * within rounding; it keeps each regression's design matrix in LDS, so it
 * needs p N + p^2 (p < N) and N p (p >= N) doubles to fit in 160 KiB.
 * Errors: EINVAL, ESTATE (no workspace), ENOTSPD, ENONPOS_D, EHIP,
 * ENOCONV (ENKFMC_FIT_SVD: a regression's Jacobi sweeps did not converge in
 * 40 sweeps), EUNSUPPORTED (the plain kernel's N x N Gram does not fit in
 * LDS: N > 141, in ENKFMC_FIT_PLAIN or for rows of the plain bucket; or the
 * design matrices of ENKFMC_FIT_SVD do not). */
enkfmc_status enkfmc_fit(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, double ridge,
                         int32_t mode, void *stream);

/* Local analyses and merge (eq. 10, eq. 11 per sub-domain / eq. 14, Alg. 2-3).
 * Needs the immediately preceding enkfmc_fit on the same X_b.
 * Xb: dev (n x N, dtype, ld); Y: dev (m x N) float64 perturbed observations;
 * r_diag: dev (m) float64 > 0; Xa: dev (n x N) contiguous, element type
 * out_dtype.  The local increments of all rows stay in the workspace for
 * enkfmc_analyze_backward.  solver: enkfmc_solver.  ENKFMC_SOLVE_PCG iterates
 * (Section 2.3 after eq. 13: the primal system by an iterative solver) until
 * every (block, member) column's residual, in the norm of the
 * preconditioner, is below rtol times its initial value, then recomputes
 * the residual from the solution in FP64 and restarts where it is still
 * above (enkfmc_set_pcg sets rtol and the iteration limit); it needs
 * synchronous calls (not enkfmc_set_async).
 * Errors: EINVAL, ESTATE, ENOTSPD, EHIP, ENOCONV (PCG: some column still
 * above rtol after maxit iterations; X_a then holds the last iterate and
 * the reverse pass is refused). */
enkfmc_status enkfmc_analyze(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                             const double *r_diag, void *Xa, int32_t out_dtype, int32_t solver, void *stream);

/* Reverse-mode derivative of fit + analysis.  Given dXa = dL/dX_a (dev, n x N
 * float64) it writes dL/dX_b (dev, n x N float64, overwritten), dL/dlog r
 * (dev, m float64, overwritten) and dL/dridge (dev, 1 float64, overwritten).
 * Needs the immediately preceding enkfmc_fit + enkfmc_analyze on the same
 * inputs (same Xb, Y, r_diag, ridge), else ESTATE.  Recomputes each
 * regression's Gram and factor instead of storing them, in the form (plain or
 * batched) of the preceding fit.  Sums over the overlapping halos in a fixed
 * order, so results are bitwise repeatable.  EUNSUPPORTED for N > 128. */
enkfmc_status enkfmc_analyze_backward(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                                      const double *r_diag, const double *dXa, double *dXb, double *dlogR,
                                      double *dridge, void *stream);

/* Perturbed observations of one assimilation time (Alg. 1, its
 * create_perturbed_observations step; Section 2.3 after eq. 11: the columns
 * of Y^s carry data errors drawn from N(0, R), not re-centred).
 * y: dev (m) float64 observations; r_diag: dev (m) float64 > 0;
 * Ys: dev (m x N) float64, overwritten with
 *   Ys[o][k] = y[o] + sqrt(r_diag[o]) * xi(seed, cycle, o, k).
 * xi is standard normal: the Philox4x64-10 block (Salmon et al., SC'11) with
 * key (seed, 0) and counter (k / 4, o, cycle, 0) gives four 64-bit words
 * w_0..w_3; u_i = ((w_i >> 12) + 1/2) * 2^-52; Box-Muller maps (u_0, u_1) to
 * members 4j, 4j+1 and (u_2, u_3) to 4j+2, 4j+3 (j = k / 4):
 *   z = sqrt(-2 ln u_0) cos(2 pi u_1), z' = sqrt(-2 ln u_0) sin(2 pi u_1).
 * A draw depends only on (seed, cycle, o, k).  Ys must not be the Y of an
 * analysis whose enkfmc_analyze_backward is still to come.
 * Errors: EINVAL (NULL argument), ESTATE (no workspace), EHIP. */
enkfmc_status enkfmc_perturb_observations(enkfmc_plan *p, const double *y, const double *r_diag, uint64_t seed,
                                          uint64_t cycle, double *Ys, void *stream);

/* Squared error of the analysis mean at one assimilation time, the summand
 * of the RMSE of eq. (18) (Section 4):
 *   err[0] = sum_g (mean_k Xa[g][k] - x_ref[g])^2.
 * Xa: dev (n x N), element type dtype, row stride ld >= N; x_ref: dev (n)
 * float64; err: dev (1) float64, overwritten.  The sums run in a fixed order,
 * so the result is bitwise repeatable.  Uses the workspace as scratch but
 * leaves the state of fit and analysis as it was.
 * Errors: EINVAL, ESTATE (no workspace), EHIP. */
enkfmc_status enkfmc_analysis_sq_error(enkfmc_plan *p, const void *Xa, int32_t dtype, int64_t ld,
                                       const double *x_ref, double *err, void *stream);

/* RMSE of the analysis mean over M assimilation times, eq. (18) as printed
 * (no 1/n): out[0] = sqrt((1/M) sum_t sq_err[t]), with sq_err (dev, M >= 1
 * float64) the values of enkfmc_analysis_sq_error.  One kernel, fixed-order
 * sum; only enqueued on `stream`.  Errors: EINVAL, EHIP. */
enkfmc_status enkfmc_rmse(const double *sq_err, int64_t M, double *out, void *stream);

/* The same squared error as enkfmc_analysis_sq_error, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): it needs no plan and no workspace, and
 * calls no allocating routine.  Same arguments and arithmetic (the same
 * kernels, so the same bits), with n (components) and N (members) given
 * directly.  Its scratch, the 256 partial sums of the first reduction level
 * (2 KiB), is a static device array that every GPU the library runs on holds
 * until the process ends; it does not grow with n.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * threads) race and must not be issued.  The call only enqueues its two
 * kernels on `stream` and returns without waiting; err is valid once the
 * stream has reached that point.
 * Limits: n <= ENKFMC_SQ_ERROR_NOALLOC_MAX_N, N <= ENKFMC_SQ_ERROR_NOALLOC_MAX_MEMBERS
 * (larger sizes return EUNSUPPORTED).
 * Errors: EINVAL (NULL pointer, bad dtype, n < 0, N < 1, ld < N),
 * EUNSUPPORTED, EHIP (launch failure or scratch lookup on this device). */
#define ENKFMC_SQ_ERROR_NOALLOC_MAX_N ((int64_t)2147483647)
#define ENKFMC_SQ_ERROR_NOALLOC_MAX_MEMBERS 65536
enkfmc_status enkfmc_analysis_sq_error_noalloc(int64_t n, int32_t N, const void *Xa, int32_t dtype, int64_t ld,
                                               const double *x_ref, double *err, void *stream);

/* Parity exports of sub-domain k (host copies, local numbering of Section 3).
 * Sizes first, then the arrays (any pointer may be NULL to skip it):
 *  loc2glob[n_sd]   global component of each local row
 *  interior[n_sd]   1 if the row is mapped back (not halo)
 *  row_ptr[n_sd+1]  CSR of the strictly-lower pattern of T
 *  col_idx[nnz_sd]  local predecessor rows, ascending within a row
 *  obs[m_sd]        observation numbers o inside the extended box, ascending
 *  obs_row[m_sd]    local row of each of them */
enkfmc_status enkfmc_get_pattern_sizes(const enkfmc_plan *p, int32_t k, int64_t *n_sd, int64_t *nnz_sd,
                                       int64_t *m_sd);
enkfmc_status enkfmc_get_pattern(const enkfmc_plan *p, int32_t k, int64_t *loc2glob, uint8_t *interior,
                                 int64_t *row_ptr, int32_t *col_idx, int32_t *obs, int32_t *obs_row);

/* Fitted factors of sub-domain k after enkfmc_fit (host copies): tval[nnz_sd]
 * = T values (= -beta) in the CSR order of enkfmc_get_pattern, d[n_sd] = D. */
enkfmc_status enkfmc_get_factors(enkfmc_plan *p, int32_t k, double *tval, double *d, void *stream);

/* Local increments Z (host, n_sd x N) of sub-domain k after enkfmc_analyze,
 * halo rows included. */
enkfmc_status enkfmc_get_increment(enkfmc_plan *p, int32_t k, double *Z, void *stream);

/* Limits of ENKFMC_SOLVE_PCG: at most maxit >= 1 iterations (default 2000),
 * relative tolerance 0 < rtol < 1 on the preconditioned residual norm
 * (default 1e-12).  Iterations run in HIP graphs of 8, so the count is a
 * multiple of 8 (a column that converges stops changing).
 * enkfmc_get_pcg_stats reports the last PCG analysis: iterations run,
 * the largest per-column count, the restarts after refinement and the
 * largest final relative residual over the columns. */
enkfmc_status enkfmc_set_pcg(enkfmc_plan *p, int32_t maxit, double rtol);
enkfmc_status enkfmc_get_pcg_stats(enkfmc_plan *p, int32_t *iterations, int32_t *max_column_iterations,
                                   int32_t *refinements, double *max_rel_residual, void *stream);

/* Asynchronous mode of a plan (enable != 0), for running many plans
 * concurrently and for capturing calls into a HIP graph: enkfmc_fit,
 * enkfmc_analyze and enkfmc_analyze_backward then only enqueue their kernels
 * (no memset, no device-to-host read, no synchronisation) and return
 * ENKFMC_OK unless an argument or launch fails.  Device-side failures
 * (ENOTSPD, ENONPOS_D, ENOCONV) accumulate in the plan's status word, first
 * failure kept, until enkfmc_check_status reads it: it synchronises `stream`,
 * returns the recorded status (with enkfmc_last_error naming the row or
 * block) and clears the word.  Phase timing is off in this mode.  The state
 * checks of the calls (fit before analyze, same inputs before the reverse
 * pass) still apply, to the enqueued order. */
enkfmc_status enkfmc_set_async(enkfmc_plan *p, int32_t enable);
enkfmc_status enkfmc_check_status(enkfmc_plan *p, void *stream);

/* Device timestamp for latency measurements: one kernel writes the device's
 * constant-rate wall clock (ticks of enkfmc_wall_clock_hz) to dev (a device
 * uint64) when the stream reaches it.  Capturable into a HIP graph. */
enkfmc_status enkfmc_timestamp(uint64_t *dev, void *stream);
enkfmc_status enkfmc_wall_clock_hz(int64_t *hz);

/* Per-phase kernel timing (HIP events recorded on the call's stream around
 * each kernel).  enable != 0 turns it on for later calls; enkfmc_get_timing
 * returns the duration in ms of phase `phase` in the most recent timed call
 * (0 if that call did not run it: every timed call clears the others).
 * Phases: */
enum {
  ENKFMC_PH_ANOMALY = 0,   /* mean and anomalies, eq. (5)                          */
  ENKFMC_PH_FIT = 1,       /* regressions, eq. (1)                                 */
  ENKFMC_PH_DUAL_F = 2,    /* F = T^-T H^T                                         */
  ENKFMC_PH_DUAL_S = 3,    /* S = R + F^T D F                                      */
  ENKFMC_PH_DUAL_CHOL = 4, /* Cholesky of S                                        */
  ENKFMC_PH_DUAL_Q = 5,    /* Q = S^-1 (Y^s - H X_b)                               */
  ENKFMC_PH_DUAL_G = 6,    /* D (F Q)                                              */
  ENKFMC_PH_SWEEP = 7,     /* Z = T^-1 (...)                                       */
  ENKFMC_PH_MAPBACK = 8,   /* X_a = X_b + Z on interior rows                       */
  ENKFMC_PH_BACKWARD = 9,  /* whole reverse pass                                   */
  ENKFMC_PH_TILES = 10,    /* dense 16x16 tiles of T and inverse diagonal tiles     */
  ENKFMC_PH_FIT_KFORM = 11, /* kernel-form regressions (p >= N) alone, within FIT  */
  ENKFMC_PH_ADJ_SOLVE = 12, /* adjoint: W = A^-1 Zbar (within BACKWARD)            */
  ENKFMC_PH_ADJ_FACTOR = 13, /* adjoint: Dbar, betabar (within BACKWARD)           */
  ENKFMC_PH_ADJ_REGRESS = 14, /* adjoint of the regressions (within BACKWARD)      */
  ENKFMC_PH_ADJ_GATHER = 15, /* adjoint: halo gathers, dlog r, dlam (within BACKWARD) */
  ENKFMC_PH_FIT_FALLBACK = 16, /* batched fit: rows of the plain bucket alone, within FIT */
  ENKFMC_PH_PCG = 17,      /* ENKFMC_SOLVE_PCG: the whole iteration                 */
  ENKFMC_PH_COUNT = 18
};
enkfmc_status enkfmc_set_timing(enkfmc_plan *p, int32_t enable);
enkfmc_status enkfmc_get_timing(const enkfmc_plan *p, int32_t phase, double *ms);

const char *enkfmc_status_string(int32_t status);
const char *enkfmc_last_error(void);
void enkfmc_plan_destroy(enkfmc_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* ENKFMC_H */
