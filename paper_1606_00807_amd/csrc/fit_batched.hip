// Batched FP64 modified-Cholesky fit (eq. 1 / eq. 8): one 64-lane wavefront
// per regression, everything in registers.
//
// Per regression (p predecessors, N members, ridge mu = lam*(N-1)):
//   m = N (kernel form, p >= N and lam > 0) or m = p (p-form), T = ceil(m/16).
//   1. Gram  G = X^T X (+ mu I) with X = U_P (kernel form, reduction over the
//      p predecessors) or X = U_P^T (p-form, reduction over the N members),
//      accumulated by v_mfma_f64_16x16x4 into the T(T+1)/2 lower 16x16 tiles.
//      Rows/columns m..16T-1 are padded with the identity.
//   2. An extra tile row holds the right-hand side v^T (v = u or U_P u), so
//      the Cholesky factorisation of the bordered matrix [[G, v], [v^T, .]]
//      yields y = L^-1 v in its last row (forward substitution for free).
//   3. Blocked right-looking Cholesky, panel width 16: inside a panel the 16
//      columns are eliminated one at a time (column broadcast through a
//      wavefront-private LDS buffer); the trailing tiles are then updated with
//      v_mfma_f64_16x16x4 (A and B operands transposed through LDS).
//   4. Back substitution L^T x = y, blocked: off-diagonal tiles by
//      wavefront reductions, diagonal tiles by 16 scalar steps.
//   5. p-form: beta = x, eps = u - U_P^T beta;
//      kernel form: w = x, beta = U_P w, eps = mu w.   d = eps^T eps/(N-1).
//
// Layout of a v_mfma_f64_16x16x4 accumulator (lane l = 16q + c, register r):
// element (4r + q, c).  A operand: lane l holds A[c][q]; B operand: B[q][c].
#include "device.h"

namespace enkfmc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxT = 5;          // largest tile count handled here (m <= 80)
constexpr int kMaxP = 128;        // largest predecessor count handled here
constexpr int kTileLd = 17;       // padded row stride of the transpose buffer

struct WaveLds {                  // wavefront-private LDS (doubles unless noted)
  int pidx[kMaxP];
  double col[16 * (kMaxT + 1)];
  double vec[16 * (kMaxT + 1)];
  double tile[(kMaxT + 1) * 16 * kTileLd];
};

__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

__device__ inline double readlane_d(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders this wavefront's LDS accesses (LDS executes a wavefront's operations
// in issue order; this keeps the compiler from moving them).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int T>
__device__ __forceinline__ constexpr int tix(int I, int J) {  // lower tile (I >= J, I < T); aug row I == T
  return I < T ? I * (I + 1) / 2 + J : T * (T + 1) / 2 + J;
}

template <int T>
__device__ __forceinline__ void fit_row(const int lane, const int64_t r, const int p, const int N, const bool kform, const double mu,
                        const double *__restrict__ U, const int ldu, const double *__restrict__ u, WaveLds &L,
                        double *__restrict__ tval, const int64_t lo, double *__restrict__ dvec, int32_t *status) {
  constexpr int NT = T * (T + 1) / 2;
  const int q = lane >> 4, c = lane & 15;
  const int m = kform ? N : p;
  d4 acc[NT + T];
#pragma unroll
  for (int t = 0; t < NT + T; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  // ---- 1. Gram -------------------------------------------------------------
  const int K = kform ? p : N;
  const int ksteps = (K + 3) >> 2;
  for (int ks = 0; ks < ksteps; ++ks) {
    double f[T];
    if (kform) {
      const int k = 4 * ks + q;
      const int kk = k < p ? k : p - 1;
      const double *src = U + (int64_t)L.pidx[kk] * ldu;
#pragma unroll
      for (int I = 0; I < T; ++I) {
        const double x = src[16 * I + c];
        f[I] = k < p ? x : 0.0;
      }
    } else {
      const int k = 4 * ks + q;
#pragma unroll
      for (int I = 0; I < T; ++I) {
        const int a = 16 * I + c;
        const int aa = a < p ? a : p - 1;
        const double x = U[(int64_t)L.pidx[aa] * ldu + k];
        f[I] = a < p ? x : 0.0;
      }
    }
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
      for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(f[I], f[J], acc[tix<T>(I, J)]);
  }
  // ridge on the diagonal, identity on the padding
#pragma unroll
  for (int J = 0; J < T; ++J)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
      if (4 * rr + q == c) {
        const int idx = 16 * J + c;
        acc[tix<T>(J, J)][rr] = idx < m ? acc[tix<T>(J, J)][rr] + mu : 1.0;
      }
  // ---- 2. right-hand side in row 0 of the extra tile row -------------------
  if (!kform) {
    for (int a = lane; a < p; a += 64) {
      const double *ua = U + (int64_t)L.pidx[a] * ldu;
      double s = 0.0;
      for (int cc = 0; cc < N; ++cc) s += ua[cc] * u[cc];
      L.vec[a] = s;
    }
    wave_lds_sync();
  }
  if (q == 0) {
#pragma unroll
    for (int J = 0; J < T; ++J) {
      const int idx = 16 * J + c;
      const double v = kform ? u[idx] : L.vec[idx < p ? idx : 0];
      acc[tix<T>(T, J)][0] = idx < m ? v : 0.0;
    }
  }
  wave_lds_sync();

  // ---- 3. blocked Cholesky of the bordered matrix -------------------------
#pragma unroll
  for (int J = 0; J < T; ++J) {
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int qk = kk & 3, rk = kk >> 2;
      const double piv = readlane_d(acc[tix<T>(J, J)][rk], 16 * qk + kk);
      if (!(piv > 0.0)) {
        if (lane == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
        return;
      }
      const double lkk = sqrt(piv);
      const double inv = 1.0 / lkk;
      if (c == kk) {
#pragma unroll
        for (int I = J; I <= T; ++I) {
          d4 v = acc[tix<T>(I, J)];
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) v[rr] = (I == J && 4 * rr + q == kk) ? lkk : v[rr] * inv;
          acc[tix<T>(I, J)] = v;
          *(d4 *)&L.col[16 * I + 4 * q] = v;   // element (16I + 4rr + q) stored at 16I + 4q + rr
        }
      }
      wave_lds_sync();
      const double colv = L.col[16 * J + 4 * (c & 3) + (c >> 2)];
      const double cv = c > kk ? colv : 0.0;
#pragma unroll
      for (int I = J; I <= T; ++I) {
        const d4 rowv = *(const d4 *)&L.col[16 * I + 4 * q];
        d4 v = acc[tix<T>(I, J)];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) v[rr] -= rowv[rr] * cv;
        acc[tix<T>(I, J)] = v;
      }
      wave_lds_sync();
    }
    if (J + 1 < T) {
      // transpose the panel tiles below the diagonal into LDS (row-major, padded)
#pragma unroll
      for (int I = J + 1; I <= T; ++I) {
        double *tb = L.tile + (I - J - 1) * 16 * kTileLd;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) tb[(4 * rr + q) * kTileLd + c] = acc[tix<T>(I, J)][rr];
      }
      wave_lds_sync();
#pragma unroll
      for (int I2 = J + 1; I2 < T; ++I2) {
        const double *tb2 = L.tile + (I2 - J - 1) * 16 * kTileLd;
        double fb[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) fb[kc] = tb2[c * kTileLd + 4 * kc + q];
#pragma unroll
        for (int I = I2; I <= T; ++I) {
          const double *tb = L.tile + (I - J - 1) * 16 * kTileLd;
          d4 a = acc[tix<T>(I, I2)];
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) a = mfma64(-tb[c * kTileLd + 4 * kc + q], fb[kc], a);
          acc[tix<T>(I, I2)] = a;
        }
      }
      wave_lds_sync();
    }
  }

  // ---- 4. back substitution L^T x = y (y = row 0 of the extra tile row) ---
  double *y = L.vec;   // y then x, natural order
  if (q == 0) {
#pragma unroll
    for (int J = 0; J < T; ++J) y[16 * J + c] = acc[tix<T>(T, J)][0];
  }
  wave_lds_sync();
#pragma unroll
  for (int J = T - 1; J >= 0; --J) {
    double s = 0.0;
#pragma unroll
    for (int I = J + 1; I < T; ++I) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) s += acc[tix<T>(I, J)][rr] * y[16 * I + 4 * rr + q];
    }
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    double t = y[16 * J + c] - s;        // replicated over q
    // diagonal tile row-major into LDS: element (i, j) at i*17 + j
    double *tb = L.tile;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) tb[(4 * rr + q) * kTileLd + c] = acc[tix<T>(J, J)][rr];
    wave_lds_sync();
    double lrow[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) lrow[jj] = tb[jj * kTileLd + c];   // L_JJ(jj, c)
    double xc = 0.0;
#pragma unroll
    for (int jj = 15; jj >= 0; --jj) {
      const double ljj = tb[jj * kTileLd + jj];
      const double xj = readlane_d(t, jj) / ljj;
      if (c == jj) xc = xj;
      if (c < jj) t -= lrow[jj] * xj;
    }
    wave_lds_sync();
    if (q == 0) y[16 * J + c] = xc;   // x_J overwrites y_J (no longer needed)
    wave_lds_sync();
  }

  // ---- 5. coefficients and residual variance --------------------------------
  double ss = 0.0;
  if (kform) {
    for (int a = lane; a < p; a += 64) {
      const double *ua = U + (int64_t)L.pidx[a] * ldu;
      double b = 0.0;
      for (int cc = 0; cc < N; ++cc) b += ua[cc] * y[cc];
      tval[lo + a] = -b;
    }
    for (int cc = lane; cc < N; cc += 64) {
      const double e = mu * y[cc];
      ss += e * e;
    }
  } else {
    for (int a = lane; a < p; a += 64) tval[lo + a] = -y[a];
    for (int cc = lane; cc < N; cc += 64) {
      double e = u[cc];
      for (int a = 0; a < p; ++a) e -= y[a] * U[(int64_t)L.pidx[a] * ldu + cc];
      ss += e * e;
    }
  }
  ss = wave_sum(ss);
  if (lane == 0) {
    const double dd = ss / (N - 1);
    dvec[r] = dd;
    if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
  }
}

__global__ __launch_bounds__(256, 2) void k_fit_batched(const Block *__restrict__ blocks,
                                                     const int32_t *__restrict__ fit_glob,
                                                     const int32_t *__restrict__ fit_blk,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const double *__restrict__ U,
                                                     int ldu, int N, int64_t n_fit, double lam,
                                                     double *__restrict__ tval, double *__restrict__ dvec,
                                                     int32_t *status) {
  __shared__ WaveLds lds[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + wave;
  if (r >= n_fit) return;
  WaveLds &L = lds[wave];
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const double *u = U + (int64_t)fit_glob[r] * ldu;
  const double mu = lam * (double)(N - 1);
  for (int k = lane; k < p; k += 64) L.pidx[k] = fit_glob[B.row0 + col[lo + k]];
  wave_lds_sync();
  if (p == 0) {
    double s = 0.0;
    for (int cc = lane; cc < N; cc += 64) s += u[cc] * u[cc];
    s = wave_sum(s);
    if (lane == 0) {
      const double dd = s / (N - 1);
      dvec[r] = dd;
      if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
    }
    return;
  }
  const bool kform = lam > 0.0 && p >= N;
  if (!kform && lam == 0.0 && p >= N - 1) {
    if (lane == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }
  const int m = kform ? N : p;
  const int T = (m + 15) >> 4;
  switch (T) {
    case 1: fit_row<1>(lane, r, p, N, kform, mu, U, ldu, u, L, tval, lo, dvec, status); break;
    case 2: fit_row<2>(lane, r, p, N, kform, mu, U, ldu, u, L, tval, lo, dvec, status); break;
    case 3: fit_row<3>(lane, r, p, N, kform, mu, U, ldu, u, L, tval, lo, dvec, status); break;
    case 4: fit_row<4>(lane, r, p, N, kform, mu, U, ldu, u, L, tval, lo, dvec, status); break;
    default: fit_row<5>(lane, r, p, N, kform, mu, U, ldu, u, L, tval, lo, dvec, status); break;
  }
}

size_t fit_plain_lds(const enkfmc_plan *p);

hipError_t launch_fit_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  // rows whose system exceeds 80 (N > 80 in the kernel form) or with more
  // than 128 predecessors are outside this kernel's register budget
  if (p->N > 16 * kMaxT || p->max_p > kMaxP) return launch_fit_plain(p, d, lam, s);
  phase_begin(p, ENKFMC_PH_FIT, s);
  hipLaunchKernelGGL(k_fit_batched, dim3((unsigned)((p->n_fit + 3) / 4)), dim3(256), 0, s, d.blocks, d.fit_glob,
                     d.fit_blk, d.row_ptr, d.col, d.U, p->ldu, p->N, p->n_fit, lam, d.tval, d.dvec, d.status);
  phase_end(p, ENKFMC_PH_FIT, s);
  return hipGetLastError();
}

}  // namespace enkfmc
