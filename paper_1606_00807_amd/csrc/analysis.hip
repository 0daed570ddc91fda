// Local analysis of every (sub-domain, variable) block and the merge.
//
// The local primal system of eq. (11) (per sub-domain, eq. 14 / Alg. 3),
//   (T^T D^-1 T + H^T R^-1 H) Z = H^T R^-1 Delta,   Delta = Y^s - H X_b,
// is solved exactly through the dual form of eqs. (12)-(13):
//   B^ = T^-1 D T^-T,   F = T^-T H^T            (n_b x m_b, one backward sweep)
//   S  = R + H B^ H^T = R + F^T D F             (m_b x m_b, Cholesky)
//   Q  = S^-1 Delta                             (m_b x N)
//   Z  = B^ H^T Q = T^-1 (D (F Q))              (one forward sweep, N columns)
// Then X_a = X_b + Z on interior rows only (Alg. 2 merge; the interiors of
// the sub-domains do not intersect, so every component is written once).
#include "device.h"

namespace enkfmc {

// F = T^-T H^T: column o solves T^T f = e_{j_o} backwards (pull form over the
// transposed pattern).  One lane per observation column; rows sequential.
__global__ __launch_bounds__(64) void k_dual_F(const Block *__restrict__ blocks, const int64_t *__restrict__ csc_ptr,
                                               const int32_t *__restrict__ csc_row,
                                               const int32_t *__restrict__ csc_nz,
                                               const int32_t *__restrict__ bobs_row,
                                               const double *__restrict__ tval, double *__restrict__ F) {
  const Block B = blocks[blockIdx.x];
  const int o = blockIdx.y * 64 + threadIdx.x;
  if (o >= B.m) return;
  const int j = bobs_row[B.obs0 + o];
  const int mb = B.m;
  double *Fb = F + B.F0;
  const double *tv = tval + B.nz0;
  for (int q = B.n - 1; q >= 0; --q) {
    double acc = (q == j) ? 1.0 : 0.0;
    const int64_t c0 = csc_ptr[B.row0 + q], c1 = csc_ptr[B.row0 + q + 1];
    for (int64_t t = c0; t < c1; ++t) acc -= tv[csc_nz[t]] * Fb[(int64_t)csc_row[t] * mb + o];
    Fb[(int64_t)q * mb + o] = acc;
  }
}

// S = R + F^T D F (lower triangle).
__global__ __launch_bounds__(256) void k_dual_S(const Block *__restrict__ blocks, const int32_t *__restrict__ bobs_o,
                                                const double *__restrict__ F, const double *__restrict__ dvec,
                                                const double *__restrict__ r_diag, double *__restrict__ S) {
  const Block B = blocks[blockIdx.x];
  const int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int mb = B.m;
  if (idx >= (int64_t)mb * mb) return;
  const int a = (int)(idx / mb), b = (int)(idx % mb);
  if (b > a) return;
  const double *Fb = F + B.F0;
  const double *d = dvec + B.row0;
  double s = 0.0;
  for (int q = 0; q < B.n; ++q) s += (Fb[(int64_t)q * mb + a] * d[q]) * Fb[(int64_t)q * mb + b];
  if (a == b) s += r_diag[bobs_o[B.obs0 + a]];
  S[B.S0 + (int64_t)a * mb + b] = s;
}

// In-place Cholesky of each block's S (lower triangle), one workgroup per block.
__global__ __launch_bounds__(256) void k_dual_chol(const Block *__restrict__ blocks, double *__restrict__ S,
                                                   int32_t *status) {
  __shared__ int bad;
  const Block B = blocks[blockIdx.x];
  const int m = B.m, tid = threadIdx.x;
  double *L = S + B.S0;
  if (tid == 0) bad = 0;
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    if (tid == 0) {
      const double piv = L[(int64_t)k * m + k];
      if (!(piv > 0.0)) bad = 1;
      else L[(int64_t)k * m + k] = sqrt(piv);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) set_error(status, ENKFMC_ENOTSPD, -1 - (int32_t)blockIdx.x);
      return;
    }
    const double lkk = L[(int64_t)k * m + k];
    for (int i = k + 1 + tid; i < m; i += 256) L[(int64_t)i * m + k] /= lkk;
    __syncthreads();
    const int t = m - k - 1;
    for (int64_t idx = tid; idx < (int64_t)t * t; idx += 256) {
      const int i = k + 1 + (int)(idx / t), j = k + 1 + (int)(idx % t);
      if (j <= i) L[(int64_t)i * m + j] -= L[(int64_t)i * m + k] * L[(int64_t)j * m + k];
    }
  }
}

// Q = S^-1 Delta, one lane per member column.
template <typename TX>
__global__ __launch_bounds__(64) void k_dual_Q(const Block *__restrict__ blocks, const int32_t *__restrict__ bobs_o,
                                               const int32_t *__restrict__ bobs_row,
                                               const int32_t *__restrict__ fit_glob, const double *__restrict__ S,
                                               const double *__restrict__ Y, const TX *__restrict__ Xb, int64_t ld,
                                               int N, double *__restrict__ Q) {
  const Block B = blocks[blockIdx.x];
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= N) return;
  const int m = B.m;
  const double *L = S + B.S0;
  double *q = Q + B.Q0;
  for (int a = 0; a < m; ++a) {
    const int o = bobs_o[B.obs0 + a];
    const int64_t g = fit_glob[B.row0 + bobs_row[B.obs0 + a]];
    double acc = Y[(int64_t)o * N + c] - (double)Xb[g * ld + c];
    for (int b = 0; b < a; ++b) acc -= L[(int64_t)a * m + b] * q[(int64_t)b * N + c];
    q[(int64_t)a * N + c] = acc / L[(int64_t)a * m + a];
  }
  for (int a = m - 1; a >= 0; --a) {
    double acc = q[(int64_t)a * N + c];
    for (int b = a + 1; b < m; ++b) acc -= L[(int64_t)b * m + a] * q[(int64_t)b * N + c];
    q[(int64_t)a * N + c] = acc / L[(int64_t)a * m + a];
  }
}

// Z rows = D (F Q)   (right-hand side of the final forward sweep).
__global__ __launch_bounds__(256) void k_dual_G(const Block *__restrict__ blocks, const double *__restrict__ F,
                                                const double *__restrict__ Q, const double *__restrict__ dvec, int N,
                                                double *__restrict__ Z) {
  const Block B = blocks[blockIdx.x];
  const int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (idx >= (int64_t)B.n * N) return;
  const int q = (int)(idx / N), c = (int)(idx % N);
  const int mb = B.m;
  const double *Fr = F + B.F0 + (int64_t)q * mb;
  const double *Qb = Q + B.Q0;
  double s = 0.0;
  for (int a = 0; a < mb; ++a) s += Fr[a] * Qb[(int64_t)a * N + c];
  Z[(B.row0 + q) * N + c] = dvec[B.row0 + q] * s;
}

// Z = T^-1 Z in place (forward sweep), one lane per member column.
__global__ __launch_bounds__(64) void k_fwd_sweep(const Block *__restrict__ blocks, const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col, const double *__restrict__ tval,
                                                  int N, double *__restrict__ Z) {
  const Block B = blocks[blockIdx.x];
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= N) return;
  double *Zb = Z + B.row0 * N;
  for (int i = 0; i < B.n; ++i) {
    double acc = Zb[(int64_t)i * N + c];
    const int64_t k0 = row_ptr[B.row0 + i], k1 = row_ptr[B.row0 + i + 1];
    for (int64_t k = k0; k < k1; ++k) acc -= tval[k] * Zb[(int64_t)col[k] * N + c];
    Zb[(int64_t)i * N + c] = acc;
  }
}

// X_a = X_b + Z on interior rows (each component has exactly one source row).
template <typename TX, typename TO>
__global__ __launch_bounds__(256) void k_mapback(const TX *__restrict__ Xb, int64_t ld,
                                                 const int32_t *__restrict__ src, const double *__restrict__ Z,
                                                 int64_t n, int N, TO *__restrict__ Xa) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * N) return;
  const int64_t g = idx / N;
  const int c = (int)(idx % N);
  Xa[idx] = (TO)((double)Xb[g * ld + c] + Z[(int64_t)src[g] * N + c]);
}

template <typename TX>
static hipError_t analysis_typed(enkfmc_plan *p, const Dev &d, const TX *Xb, int64_t ld, const double *Y,
                                 const double *r_diag, void *Xa, int32_t out_dtype, hipStream_t s) {
  const unsigned nb = (unsigned)p->blocks.size();
  const int N = p->N;
  if (p->max_bm > 0) {
    phase_begin(p, ENKFMC_PH_DUAL_F, s);
    hipLaunchKernelGGL(k_dual_F, dim3(nb, (p->max_bm + 63) / 64), dim3(64), 0, s, d.blocks, d.csc_ptr, d.csc_row,
                       d.csc_nz, d.bobs_row, d.tval, d.F);
    phase_end(p, ENKFMC_PH_DUAL_F, s);
    const int64_t sq = (int64_t)p->max_bm * p->max_bm;
    phase_begin(p, ENKFMC_PH_DUAL_S, s);
    hipLaunchKernelGGL(k_dual_S, dim3(nb, (unsigned)((sq + 255) / 256)), dim3(256), 0, s, d.blocks, d.bobs_o, d.F,
                       d.dvec, r_diag, d.S);
    phase_end(p, ENKFMC_PH_DUAL_S, s);
    phase_begin(p, ENKFMC_PH_DUAL_CHOL, s);
    hipLaunchKernelGGL(k_dual_chol, dim3(nb), dim3(256), 0, s, d.blocks, d.S, d.status);
    phase_end(p, ENKFMC_PH_DUAL_CHOL, s);
    phase_begin(p, ENKFMC_PH_DUAL_Q, s);
    hipLaunchKernelGGL(k_dual_Q<TX>, dim3(nb, (N + 63) / 64), dim3(64), 0, s, d.blocks, d.bobs_o, d.bobs_row,
                       d.fit_glob, d.S, Y, Xb, ld, N, d.Q);
    phase_end(p, ENKFMC_PH_DUAL_Q, s);
  }
  const int64_t nbN = (int64_t)p->max_bn * N;
  phase_begin(p, ENKFMC_PH_DUAL_G, s);
    hipLaunchKernelGGL(k_dual_G, dim3(nb, (unsigned)((nbN + 255) / 256)), dim3(256), 0, s, d.blocks, d.F, d.Q, d.dvec, N,
                     d.Z);
    phase_end(p, ENKFMC_PH_DUAL_G, s);
  phase_begin(p, ENKFMC_PH_SWEEP, s);
    hipLaunchKernelGGL(k_fwd_sweep, dim3(nb, (N + 63) / 64), dim3(64), 0, s, d.blocks, d.row_ptr, d.col, d.tval, N, d.Z);
    phase_end(p, ENKFMC_PH_SWEEP, s);
  const int64_t tot = p->n * N;
  const dim3 g((unsigned)((tot + 255) / 256));
  phase_begin(p, ENKFMC_PH_MAPBACK, s);
  if (out_dtype == ENKFMC_F32)
    hipLaunchKernelGGL((k_mapback<TX, float>), g, dim3(256), 0, s, Xb, ld, d.interior_src, d.Z, p->n, N, (float *)Xa);
  else
    hipLaunchKernelGGL((k_mapback<TX, double>), g, dim3(256), 0, s, Xb, ld, d.interior_src, d.Z, p->n, N,
                       (double *)Xa);
  phase_end(p, ENKFMC_PH_MAPBACK, s);
  return hipGetLastError();
}

hipError_t launch_analysis_dual(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld,
                                const double *Y, const double *r_diag, void *Xa, int32_t out_dtype, hipStream_t s) {
  if (dtype == ENKFMC_F32) return analysis_typed(p, d, (const float *)Xb, ld, Y, r_diag, Xa, out_dtype, s);
  return analysis_typed(p, d, (const double *)Xb, ld, Y, r_diag, Xa, out_dtype, s);
}

}  // namespace enkfmc
