// Ensemble anomalies (eq. 5) and the plain FP64 modified-Cholesky fit
// (eq. 1 / eq. 8): one 256-thread workgroup per regression, Gram and
// Cholesky factor in LDS.
//
// Regression of row i on its p predecessors P (ridge mu = lam*(N-1) on the
// un-normalised Gram, identical to lam on the (N-1)-normalised one):
//   p-form (p < N, or lam == 0):  (U_P U_P^T + mu I) beta = U_P u,
//                                  eps = u - U_P^T beta
//   kernel form (p >= N, lam > 0): (U_P^T U_P + mu I) w = u, beta = U_P w,
//                                  eps = mu w          (push-through identity)
//   d = eps^T eps / (N-1);  T_{i,P} = -beta.
// The kernel form factors an N x N instead of a p x p matrix; it needs
// lam > 0 because U_P^T U_P annihilates the all-ones vector.
#include "device.h"

namespace enkfmc {

template <typename TX>
__global__ __launch_bounds__(256) void k_anomaly(const TX *__restrict__ Xb, int64_t ld, int64_t n, int N, int ldu,
                                                 double *__restrict__ mean, double *__restrict__ U) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= n + 2) return;
  if (row >= n) {  // zero pad rows after the n anomaly rows
    for (int c = lane; c < ldu; c += 64) U[row * ldu + c] = 0.0;
    return;
  }
  const TX *x = Xb + row * ld;
  double s = 0.0;
  for (int c = lane; c < N; c += 64) s += (double)x[c];
  s = wave_sum(s);
  const double mu = s / N;
  if (lane == 0) mean[row] = mu;
  double *u = U + row * ldu;
  for (int c = lane; c < ldu; c += 64) u[c] = c < N ? (double)x[c] - mu : 0.0;
}

hipError_t launch_anomaly(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, hipStream_t s) {
  const dim3 grid((unsigned)((p->n + 2 + 3) / 4)), block(256);
  phase_begin(p, ENKFMC_PH_ANOMALY, s);
  if (dtype == ENKFMC_F32)
    hipLaunchKernelGGL(k_anomaly<float>, grid, block, 0, s, (const float *)Xb, ld, p->n, p->N, p->ldu, d.mean, d.U);
  else
    hipLaunchKernelGGL(k_anomaly<double>, grid, block, 0, s, (const double *)Xb, ld, p->n, p->N, p->ldu, d.mean,
                       d.U);
  phase_end(p, ENKFMC_PH_ANOMALY, s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fit_plain(const Block *__restrict__ blocks,
                                                   const int32_t *__restrict__ fit_glob,
                                                   const int32_t *__restrict__ fit_blk,
                                                   const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col, const double *__restrict__ U,
                                                   int ldu, int N, int max_p, double lam, double *__restrict__ tval,
                                                   double *__restrict__ dvec, int32_t *status,
                                                   const int32_t *__restrict__ rows) {
  extern __shared__ double smem[];
  __shared__ int bad;
  const int64_t r = rows ? (int64_t)rows[blockIdx.x] : (int64_t)blockIdx.x;
  const int tid = threadIdx.x;
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const double *u = U + (int64_t)fit_glob[r] * ldu;
  const double mu = lam * (double)(N - 1);
  const bool kform = lam > 0.0 && p >= N;
  const int m = kform ? N : p;
  double *G = smem;                                 // N*N
  double *v = G + (size_t)N * N;                    // max(N, max_p)
  double *red = v + (N > max_p ? N : max_p);        // 8
  int *pidx = (int *)(red + 8);                     // max_p
  if (tid == 0) bad = 0;
  for (int k = tid; k < p; k += 256) pidx[k] = fit_glob[B.row0 + col[lo + k]];
  __syncthreads();
  if (p == 0) {
    double s = 0.0;
    for (int c = tid; c < N; c += 256) s += u[c] * u[c];
    s = block_sum256(s, red);
    if (tid == 0) {
      const double dd = s / (N - 1);
      dvec[r] = dd;
      if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
    }
    return;
  }
  if (!kform && lam == 0.0 && p >= N - 1) {
    if (tid == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }
  // Gram (lower triangle) and right-hand side
  if (kform) {
    for (int idx = tid; idx < m * m; idx += 256) {
      const int a = idx / m, b = idx % m;
      if (b > a) continue;
      double s = 0.0;
      for (int q = 0; q < p; ++q) {
        const double *uq = U + (int64_t)pidx[q] * ldu;
        s += uq[a] * uq[b];
      }
      G[a * m + b] = s + (a == b ? mu : 0.0);
    }
    for (int a = tid; a < m; a += 256) v[a] = u[a];
  } else {
    for (int idx = tid; idx < m * m; idx += 256) {
      const int a = idx / m, b = idx % m;
      if (b > a) continue;
      const double *ua = U + (int64_t)pidx[a] * ldu, *ub = U + (int64_t)pidx[b] * ldu;
      double s = 0.0;
      for (int c = 0; c < N; ++c) s += ua[c] * ub[c];
      G[a * m + b] = s + (a == b ? mu : 0.0);
    }
    for (int a = tid; a < m; a += 256) {
      const double *ua = U + (int64_t)pidx[a] * ldu;
      double s = 0.0;
      for (int c = 0; c < N; ++c) s += ua[c] * u[c];
      v[a] = s;
    }
  }
  __syncthreads();
  // right-looking Cholesky, lower triangle in place
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      const double piv = G[k * m + k];
      if (!(piv > 0.0)) bad = 1;
      else G[k * m + k] = sqrt(piv);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
      return;
    }
    const double lkk = G[k * m + k];
    for (int i = k + 1 + tid; i < m; i += 256) G[i * m + k] /= lkk;
    __syncthreads();
    const int t = m - k - 1;
    for (int idx = tid; idx < t * t; idx += 256) {
      const int i = k + 1 + idx / t, j = k + 1 + idx % t;
      if (j <= i) G[i * m + j] -= G[i * m + k] * G[j * m + k];
    }
    __syncthreads();
  }
  // L y = v, then L^T x = y
  for (int k = 0; k < m; ++k) {
    if (tid == 0) v[k] /= G[k * m + k];
    __syncthreads();
    const double yk = v[k];
    for (int i = k + 1 + tid; i < m; i += 256) v[i] -= G[i * m + k] * yk;
    __syncthreads();
  }
  for (int k = m - 1; k >= 0; --k) {
    if (tid == 0) v[k] /= G[k * m + k];
    __syncthreads();
    const double xk = v[k];
    for (int i = tid; i < k; i += 256) v[i] -= G[k * m + i] * xk;
    __syncthreads();
  }
  double s = 0.0;
  if (kform) {
    for (int a = tid; a < p; a += 256) {
      const double *ua = U + (int64_t)pidx[a] * ldu;
      double b = 0.0;
      for (int c = 0; c < N; ++c) b += ua[c] * v[c];
      tval[lo + a] = -b;
    }
    for (int c = tid; c < N; c += 256) {
      const double e = mu * v[c];
      s += e * e;
    }
  } else {
    for (int a = tid; a < p; a += 256) tval[lo + a] = -v[a];
    for (int c = tid; c < N; c += 256) {
      double e = u[c];
      for (int a = 0; a < p; ++a) e -= v[a] * U[(int64_t)pidx[a] * ldu + c];
      s += e * e;
    }
  }
  s = block_sum256(s, red);
  if (tid == 0) {
    const double dd = s / (N - 1);
    dvec[r] = dd;
    if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
  }
}

size_t fit_plain_lds(const enkfmc_plan *p) {
  const int N = p->N, mp = p->max_p;
  return (size_t)N * N * 8 + (size_t)(N > mp ? N : mp) * 8 + 8 * 8 + (size_t)mp * 4 + 16;
}

bool fit_plain_fits(const enkfmc_plan *p) { return fit_plain_lds(p) <= 160 * 1024; }

// The plain kernel over a list of fit rows (every row when rows is NULL).
hipError_t launch_fit_plain_rows(enkfmc_plan *p, const Dev &d, double lam, const int32_t *rows, int64_t nrows,
                                 hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const size_t lds = fit_plain_lds(p);
  hipError_t e = hipFuncSetAttribute((const void *)k_fit_plain, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fit_plain, dim3((unsigned)nrows), dim3(256), lds, s, d.blocks, d.fit_glob, d.fit_blk,
                     d.row_ptr, d.col, d.U, p->ldu, p->N, p->max_p, lam, d.tval, d.dvec, d.status, rows);
  return hipGetLastError();
}

hipError_t launch_fit_plain(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  phase_begin(p, ENKFMC_PH_FIT, s);
  const hipError_t e = launch_fit_plain_rows(p, d, lam, nullptr, p->n_fit, s);
  phase_end(p, ENKFMC_PH_FIT, s);
  return e;
}

}  // namespace enkfmc
