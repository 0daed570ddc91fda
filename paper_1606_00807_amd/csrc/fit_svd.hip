// The regressions of eq. (1) by the singular value decomposition of their
// design matrices, the route Section 5 proposes for accelerators: one
// 256-thread workgroup per regression, one-sided (Hestenes) Jacobi in LDS.
//
// Row i with predecessors P (p of them), anomalies u = u_i, ridge
// mu = lam (N - 1) on the un-normalised Gram.  With A = U_P^T (N x p) =
// W diag(sigma) V^T, the ridge solution is beta = V diag(sigma/(sigma^2 + mu)) W^T u.
// Jacobi rotates the columns of a matrix M until they are mutually
// orthogonal, M G_1 G_2 ... = M V; the columns of M V are then W diag(sigma),
// and sigma_j^2 is the squared norm of column j.
//
//   p-form (p < N, or lam == 0): M = A, p columns of length N.  V (p x p) is
//     accumulated from the rotations, y_j = (M V)_j . u / (sigma_j^2 + mu),
//     beta = V y.  With lam == 0 a zero singular value is ENOTSPD.
//   kernel form (p >= N, lam > 0): M = U_P = A^T, N columns of length p.  Here
//     M V = Q diag(sigma) gives A = V diag(sigma) Q^T, so
//     beta = Q diag(sigma/(sigma^2 + mu)) V^T u = sum_j (M V)_j z_j/(sigma_j^2 + mu)
//     with z = V^T u, which the rotations update directly (no V needed).
//
// Both forms then take eps = u - U_P^T beta and d = eps^T eps / (N - 1), as
// the Cholesky fit does.
//
// Rotations: the pairs of one round of a round-robin ordering are disjoint,
// so the 16-lane groups of the workgroup (16 of them) take different pairs at
// once; a group sums the pair's three inner products over its 16 lanes.  A
// pair (a, b) with alpha = |m_a|^2, beta = |m_b|^2, gamma = m_a . m_b is
// rotated when |gamma| > tol sqrt(alpha beta), tol = L 2^-53:
//   zeta = (beta - alpha)/(2 gamma), t = sign(zeta)/(|zeta| + sqrt(1 + zeta^2)),
//   c = 1/sqrt(1 + t^2), s = c t,
//   m_a <- c m_a - s m_b,  m_b <- s m_a + c m_b   (the same on V or on z),
// which makes the new inner product zero.  Sweeps repeat until one makes no
// rotation; a regression still rotating after kSvdMaxSweeps sweeps is ENOCONV.
#include <algorithm>

#include "device.h"

namespace enkfmc {
namespace {

constexpr int kSvdMaxSweeps = 40;

// Sum over each row of 16 lanes (every lane of the row gets it).  Partner
// lanes i^1, i^2 inside quads, then the mirrored lane in the half row and in
// the row.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double sum16(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// Column at position pos of round rd of the round-robin ordering of cp
// (even) columns: position 0 stays, the others turn by one place per round.
__device__ __forceinline__ int rr_col(int pos, int rd, int cp) {
  return pos == 0 ? 0 : 1 + (pos - 1 + rd) % (cp - 1);
}

// LDS carve-up of one regression (doubles, then the int predecessor list).
struct SvdLds {
  int c, L, Ls;            // columns, their length, column stride
  size_t m, v, u, w, beta, pidx, total_bytes;
};

__host__ __device__ inline SvdLds svd_lds(int p, int N, bool kform) {
  SvdLds s{};
  s.c = kform ? N : p;
  s.L = kform ? p : N;
  s.Ls = s.L;
  size_t off = 0;
  s.m = off; off += (size_t)s.c * s.Ls;
  s.v = off; off += kform ? (size_t)N : (size_t)s.c * s.c;   // z (kernel form) or V
  s.u = off; off += (size_t)N;
  s.w = off; off += (size_t)s.c;
  s.beta = off; off += (size_t)p;
  s.pidx = off;
  s.total_bytes = off * sizeof(double) + (size_t)p * sizeof(int) + 16;
  return s;
}

__global__ __launch_bounds__(256) void k_fit_svd(const Block *__restrict__ blocks,
                                                 const int32_t *__restrict__ fit_glob,
                                                 const int32_t *__restrict__ fit_blk,
                                                 const int64_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col, const double *__restrict__ U,
                                                 int ldu, int N, const int32_t *__restrict__ rows, double lam,
                                                 double *__restrict__ tval, double *__restrict__ dvec,
                                                 int32_t *status) {
  extern __shared__ double sm[];
  __shared__ double red[4];
  __shared__ int rotated, bad;
  const int64_t r = rows[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q = lane >> 4, cl = lane & 15;
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const double *ug = U + (int64_t)fit_glob[r] * ldu;
  const double mu = lam * (double)(N - 1);
  if (p == 0) {   // no predecessors: d = u^T u / (N - 1)
    double s = 0.0;
    for (int k = tid; k < N; k += 256) s = fma(ug[k], ug[k], s);
    s = block_sum256(s, red);
    if (tid == 0) {
      const double dd = s / (N - 1);
      dvec[r] = dd;
      if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
    }
    return;
  }
  if (lam == 0.0 && p >= N - 1) {   // R6: no pseudo-inverse without a ridge
    if (tid == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }
  const bool kform = lam > 0.0 && p >= N;
  const SvdLds S = svd_lds(p, N, kform);
  const int c = S.c, L = S.L, Ls = S.Ls;
  double *M = sm + S.m, *V = sm + S.v, *u = sm + S.u, *w = sm + S.w, *beta = sm + S.beta;
  int *pidx = (int *)(sm + S.pidx);
  if (tid == 0) bad = 0;
  for (int a = tid; a < p; a += 256) pidx[a] = fit_glob[B.row0 + col[lo + a]];
  for (int k = tid; k < N; k += 256) u[k] = ug[k];
  __syncthreads();
  if (kform) {
    // column j = member j: M[j][a] = U[P_a][j]; reads run along the members
    for (int idx = tid; idx < p * N; idx += 256) {
      const int a = idx / N, j = idx % N;
      M[(size_t)j * Ls + a] = U[(int64_t)pidx[a] * ldu + j];
    }
    for (int j = tid; j < N; j += 256) V[j] = u[j];   // z = V^T u with V = I
  } else {
    // column j = predecessor j: M[j][k] = U[P_j][k]
    for (int idx = tid; idx < p * N; idx += 256) {
      const int j = idx / N, k = idx % N;
      M[(size_t)j * Ls + k] = U[(int64_t)pidx[j] * ldu + k];
    }
    for (int idx = tid; idx < c * c; idx += 256) V[idx] = (idx / c == idx % c) ? 1.0 : 0.0;
  }
  __syncthreads();

  // ---- one-sided Jacobi sweeps -------------------------------------------
  const int cp = c + (c & 1);          // even count; column c is a dummy when c is odd
  const int npairs = cp / 2;
  const double tol = (double)L * 0x1p-53;
  int sweep = 0;
  for (; sweep < kSvdMaxSweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd + 1 < cp; ++rd) {
      for (int pi = 4 * wave + q; pi < npairs; pi += 16) {
        const int a = rr_col(pi, rd, cp), b = rr_col(cp - 1 - pi, rd, cp);
        if (a >= c || b >= c) continue;   // the dummy column (all 16 lanes of the group agree)
        double *Ma = M + (size_t)a * Ls, *Mb = M + (size_t)b * Ls;
        double sa = 0.0, sb = 0.0, sg = 0.0;
        for (int e = cl; e < L; e += 16) {
          const double x = Ma[e], y = Mb[e];
          sa = fma(x, x, sa);
          sb = fma(y, y, sb);
          sg = fma(x, y, sg);
        }
        sa = sum16(sa);
        sb = sum16(sb);
        sg = sum16(sg);
        if (fabs(sg) > tol * sqrt(sa * sb)) {
          const double zeta = (sb - sa) / (2.0 * sg);
          const double t = fabs(zeta) > 1e150 ? 0.5 / zeta
                                               : copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
          const double cs = 1.0 / sqrt(fma(t, t, 1.0)), sn = cs * t;
          for (int e = cl; e < L; e += 16) {
            const double x = Ma[e], y = Mb[e];
            Ma[e] = cs * x - sn * y;
            Mb[e] = sn * x + cs * y;
          }
          if (kform) {
            if (cl == 0) {
              const double za = V[a], zb = V[b];
              V[a] = cs * za - sn * zb;
              V[b] = sn * za + cs * zb;
            }
          } else {
            double *Va = V + (size_t)a * c, *Vb = V + (size_t)b * c;
            for (int e = cl; e < c; e += 16) {
              const double x = Va[e], y = Vb[e];
              Va[e] = cs * x - sn * y;
              Vb[e] = sn * x + cs * y;
            }
          }
          if (cl == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  if (sweep == kSvdMaxSweeps) {
    if (tid == 0) set_error(status, ENKFMC_ENOCONV, (int32_t)r);
    return;
  }

  // ---- coefficients --------------------------------------------------------
  // w_j = z_j/(sigma_j^2 + mu) (kernel form) or (M V)_j . u/(sigma_j^2 + mu)
  for (int j = 4 * wave + q; j < c; j += 16) {
    const double *Mj = M + (size_t)j * Ls;
    double s2 = 0.0, g = 0.0;
    for (int e = cl; e < L; e += 16) {
      s2 = fma(Mj[e], Mj[e], s2);
      if (!kform) g = fma(Mj[e], u[e], g);
    }
    s2 = sum16(s2);
    if (!kform) g = sum16(g);
    const double den = s2 + mu;
    if (cl == 0) {
      if (!(den > 0.0)) bad = 1;   // lam == 0 with a zero singular value
      w[j] = (kform ? V[j] : g) / den;
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }
  // beta_a = sum_j (M V)[a][j] w_j (kernel form) or sum_j V[a][j] w_j
  for (int a = tid; a < p; a += 256) {
    double b = 0.0;
    if (kform)
      for (int j = 0; j < c; ++j) b = fma(M[(size_t)j * Ls + a], w[j], b);
    else
      for (int j = 0; j < c; ++j) b = fma(V[(size_t)j * c + a], w[j], b);
    beta[a] = b;
    tval[lo + a] = -b;
  }
  __syncthreads();
  // eps = u - U_P^T beta, d = eps^T eps / (N - 1)
  double ss = 0.0;
  for (int k = tid; k < N; k += 256) {
    double e = u[k];
    for (int a = 0; a < p; ++a) e = fma(-beta[a], U[(int64_t)pidx[a] * ldu + k], e);
    ss = fma(e, e, ss);
  }
  ss = block_sum256(ss, red);
  if (tid == 0) {
    const double dd = ss / (N - 1);
    dvec[r] = dd;
    if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
  }
}

}  // namespace

// LDS a launch over rows of at most pmax predecessors needs (the larger of
// the two forms that can occur among them).
static size_t svd_lds_bytes(int pmax, int N, double lam) {
  size_t b = svd_lds(std::min(pmax, N - 1), N, false).total_bytes;
  if (lam > 0.0 && pmax >= N) b = std::max(b, svd_lds(pmax, N, true).total_bytes);
  return b;
}

size_t fit_svd_max_lds(const enkfmc_plan *p, double lam) { return svd_lds_bytes(p->max_p, p->N, lam); }

// Every regression through k_fit_svd, bucket by bucket so that each launch
// reserves only the LDS its rows need.
hipError_t launch_fit_svd(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  phase_begin(p, ENKFMC_PH_FIT, s);
  const int64_t *bo = p->bucket_off;
  for (int b = 0; b < kBuckets; ++b) {
    const int64_t nr = bo[b + 1] - bo[b];
    if (nr <= 0) continue;
    int pmax;
    if (b == kBucketP0) pmax = 0;
    else if (b == kBucketKF || b == kBucketPlain) pmax = p->max_p;
    else pmax = std::min(16 * b, p->max_p);   // p-form bucket of b tiles: p <= 16 b
    const size_t lds = svd_lds_bytes(pmax, p->N, lam);
    hipError_t e = hipFuncSetAttribute((const void *)k_fit_svd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fit_svd, dim3((unsigned)nr), dim3(256), lds, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr,
                       d.col, d.U, p->ldu, p->N, d.fit_rows + bo[b], lam, d.tval, d.dvec, d.status);
  }
  phase_end(p, ENKFMC_PH_FIT, s);
  return hipGetLastError();
}

}  // namespace enkfmc
