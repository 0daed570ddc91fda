// Local analysis by preconditioned conjugate gradients on the primal system
// of eq. (11) (per sub-domain, eq. 14 / Alg. 3), the iterative route Section
// 2.3 names after eq. 13:
//   A Z = H^T R^-1 Delta,   A = T^T D^-1 T + H^T R^-1 H,   Delta = Y^s - H X_b,
// one (block, member) column at a time, with the modified-Cholesky estimate
// itself as the preconditioner, M^-1 = B^ = T^-1 D T^-T (eq. 8): the
// preconditioned operator is I + B^ H^T R^-1 H, the identity plus a term of
// rank m_b, so each column converges in at most m_b + 1 steps in exact
// arithmetic.
//
// Per (block, column), standard PCG:
//   X = 0, R = B, W = M^-1 R, P = W, rho = R.W, rho0 = rho
//   repeat: Q = A P, alpha = rho / (P.Q), X += alpha P, R -= alpha Q,
//           W = M^-1 R, rho' = R.W, P = W + (rho'/rho) P, rho = rho'
//   until rho <= rtol^2 rho0 (the M^-1-norm of the residual, relative).
// After convergence the residual is recomputed from X in FP64 (R = B - A X)
// and, where its M^-1-norm still exceeds the tolerance, the iteration
// restarts from X with that residual (residual refinement).
//
// The kernels of one iteration run one 64-lane wavefront per (block, 16
// member columns), numbered so that the member tiles of a block run on one
// XCD and share its T tiles in L2.  Lane (q, c) owns column c and, in row
// tile R, rows 16R + 4r + q (the rows of its v_mfma_f64_16x16x4 accumulator);
// every vector element is read back only by the lane that wrote it, so a
// kernel needs no synchronisation beyond program order.  A wavefront whose
// columns have all converged returns at once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device.h"

namespace enkfmc {
namespace {

// Per (block, column) scalars: kScalars arrays of n_blocks * N doubles.
enum { kRho = 0, kRho0 = 1, kPQ = 2, kDone = 3, kIter = 4, kScalars = 5 };

constexpr int kPcgGraphIters = 8;       // iterations per graph launch (one status read each)
constexpr int kPcgMaxRefinements = 3;   // restarts from the recomputed FP64 residual

// Sum over the four rows of 16 lanes (every lane gets its column's total).
__device__ __forceinline__ double col_sum(double v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// True when every column this wavefront owns has converged or lies past N.
__device__ __forceinline__ bool wave_done(const double *done, int colj, int N) {
  const bool d = colj >= N || done[colj] != 0.0;
  return __all(d);
}

// hw[f] = 1/r_o at the fit row f of each local observation o, else 0.
__global__ __launch_bounds__(256) void k_pcg_zero(double *__restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = 0.0;
}
__global__ __launch_bounds__(256) void k_pcg_obs_w(const int32_t *__restrict__ bobs_o,
                                                   const int32_t *__restrict__ bobs_fit,
                                                   const double *__restrict__ r_diag, int64_t ml,
                                                   double *__restrict__ hw) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < ml) hw[bobs_fit[t]] = 1.0 / r_diag[bobs_o[t]];
}

// R = -AX (refinement) or 0 (first start), then the observed rows add the
// right-hand side B = H^T R^-1 (Y^s - H X_b): one thread per (local
// observation, member); a component is observed at most once, so no two
// threads meet.
__global__ __launch_bounds__(256) void k_pcg_neg(const double *__restrict__ AX, int64_t total,
                                                 double *__restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < total) R[i] = AX ? -AX[i] : 0.0;
}
template <typename TX>
__global__ __launch_bounds__(256) void k_pcg_rhs(const int32_t *__restrict__ bobs_o,
                                                 const int32_t *__restrict__ bobs_fit,
                                                 const int32_t *__restrict__ fit_glob, const double *__restrict__ Y,
                                                 const TX *__restrict__ Xb, int64_t ld,
                                                 const double *__restrict__ r_diag, int64_t ml, int N,
                                                 double *__restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ml * N) return;
  const int64_t t = i / N;
  const int c = (int)(i % N);
  const int o = bobs_o[t];
  const int64_t f = bobs_fit[t];
  const double delta = Y[(int64_t)o * N + c] - (double)Xb[(int64_t)fit_glob[f] * ld + c];
  R[f * N + c] += delta / r_diag[o];
}

// Yo = D^-1 T V for one block's 16 columns: row tile R gets
// V_R + L_RR V_R + sum_C T_RC V_C (L_RR the strictly lower part of the unit
// lower T_RR), divided by d row by row.
__global__ __launch_bounds__(64) void k_pcg_tv(const Block *__restrict__ blocks, int ng,
                                               const int64_t *__restrict__ rt_ptr,
                                               const int32_t *__restrict__ rt_col,
                                               const int32_t *__restrict__ rt_slot, const double *__restrict__ tiles,
                                               const double *__restrict__ tdiag, const double *__restrict__ dvec,
                                               const double *__restrict__ V, int N, const double *__restrict__ done,
                                               double *__restrict__ Yo) {
  int blk, cc;
  block_tile(ng, blk, cc);
  const Block B = blocks[blk];
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  const int coll = colok ? colj : 0;
  if (done && wave_done(done + (int64_t)blk * N, colj, N)) return;
  const double *Vb = V + B.row0 * N;
  double *Yb = Yo + B.row0 * N;
  for (int R = 0; R < B.nrt; ++R) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * R + 4 * r + q;
      acc[r] = (row < B.n && colok) ? Vb[(int64_t)row * N + colj] : 0.0;
    }
    {
      const double *Tt = tdiag + (B.rt0 + R) * 256 + c * 16 + q;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int row = 16 * R + 4 * kc + q;
        const double v = (row < B.n && colok) ? Vb[(int64_t)row * N + colj] : 0.0;
        acc = mfma64(Tt[4 * kc], v, acc);
      }
    }
    const int64_t s0 = rt_ptr[B.rt0 + R], s1 = rt_ptr[B.rt0 + R + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int C = rt_col[t];
      const double *Tt = tiles + (int64_t)rt_slot[t] * 256 + c * 16 + q;
      const double *Vc = Vb + (int64_t)(16 * C + q) * N + coll;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double v = Vc[(int64_t)(4 * kc) * N];
        acc = mfma64(Tt[4 * kc], colok ? v : 0.0, acc);
      }
    }
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * R + 4 * r + q;
        if (row < B.n) Yb[(int64_t)row * N + colj] = acc[r] / dvec[B.row0 + row];
      }
    }
  }
}

// Qo = T^T Yi + hw V for one block's 16 columns (= A V when Yi = D^-1 T V):
// column tile C gets Yi_C + L_CC^T Yi_C + sum_R T_RC^T Yi_R.  With pq set,
// also the per-column V.Qo over the block.
__global__ __launch_bounds__(64) void k_pcg_ttv(const Block *__restrict__ blocks, int ng,
                                                const int64_t *__restrict__ ct_ptr,
                                                const int32_t *__restrict__ ct_row,
                                                const int32_t *__restrict__ ct_slot, const double *__restrict__ tiles,
                                                const double *__restrict__ tdiag, const double *__restrict__ hw,
                                                const double *__restrict__ Yi, const double *__restrict__ V, int N,
                                                const double *__restrict__ done, double *__restrict__ pq,
                                                double *__restrict__ Qo) {
  int blk, cc;
  block_tile(ng, blk, cc);
  const Block B = blocks[blk];
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  if (done && wave_done(done + (int64_t)blk * N, colj, N)) return;
  const double *Yb = Yi + B.row0 * N;
  const double *Vb = V + B.row0 * N;
  double *Qb = Qo + B.row0 * N;
  double dot = 0.0;
  for (int C = 0; C < B.nrt; ++C) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * C + 4 * r + q;
      acc[r] = (row < B.n && colok) ? Yb[(int64_t)row * N + colj] : 0.0;
    }
    {
      const double *Tt = tdiag + (B.rt0 + C) * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int row = 16 * C + 4 * kc + q;
        const double y = (row < B.n && colok) ? Yb[(int64_t)row * N + colj] : 0.0;
        acc = mfma64(Tt[(4 * kc + q) * 16 + c], y, acc);
      }
    }
    const int64_t s0 = ct_ptr[B.rt0 + C], s1 = ct_ptr[B.rt0 + C + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int R = ct_row[t];
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int row = 16 * R + 4 * kc + q;
        const double y = (row < B.n && colok) ? Yb[(int64_t)row * N + colj] : 0.0;
        acc = mfma64(Tt[(4 * kc + q) * 16 + c], y, acc);
      }
    }
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * C + 4 * r + q;
        if (row < B.n) {
          const double v = Vb[(int64_t)row * N + colj];
          const double qv = fma(hw[B.row0 + row], v, acc[r]);
          Qb[(int64_t)row * N + colj] = qv;
          dot = fma(v, qv, dot);
        }
      }
    }
  }
  dot = col_sum(dot);
  if (pq && q == 0 && colok) pq[(int64_t)blk * N + colj] = dot;
}

// One PCG step of one block's 16 columns after Q = A P:
//   mode 0: alpha = rho/pq, X += alpha P, R -= alpha Q, then the rest below;
//   mode 1: first start (X = 0, R = B): rho0 = rho' and P = W;
//   mode 2: restart after a refinement (R = B - A X): rho0 kept, P = W;
// then W = T^-1 D T^-T R (backward sweep V = T^-T R into W, forward sweep
// W = T^-1 (D V) in place), rho' = R.W, P = W + (rho'/rho) P, and a column
// is done once rho' <= tol2 rho0.  A wavefront with a column still going
// counts itself in *notdone.
__global__ __launch_bounds__(64) void k_pcg_step(const Block *__restrict__ blocks, int ng,
                                                 const int64_t *__restrict__ rt_ptr,
                                                 const int32_t *__restrict__ rt_col,
                                                 const int32_t *__restrict__ rt_slot,
                                                 const int64_t *__restrict__ ct_ptr,
                                                 const int32_t *__restrict__ ct_row,
                                                 const int32_t *__restrict__ ct_slot, const double *__restrict__ tiles,
                                                 const double *__restrict__ tinv, const double *__restrict__ dvec,
                                                 int N, int64_t nbN, int mode, double tol2, double *__restrict__ X,
                                                 double *__restrict__ Rv, double *__restrict__ P,
                                                 const double *__restrict__ Q, double *__restrict__ W,
                                                 double *__restrict__ sc, int32_t *__restrict__ notdone) {
  int blk, cc;
  block_tile(ng, blk, cc);
  const Block B = blocks[blk];
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  const int coll = colok ? colj : 0;
  const int64_t si = (int64_t)blk * N + coll;
  double *rho_a = sc + kRho * nbN, *rho0_a = sc + kRho0 * nbN, *pq_a = sc + kPQ * nbN;
  double *done_a = sc + kDone * nbN, *it_a = sc + kIter * nbN;
  if (mode == 0 && wave_done(done_a + (int64_t)blk * N, colj, N)) return;
  const bool active = colok && (mode != 0 || done_a[si] == 0.0);
  const int64_t off = B.row0 * N;
  double *Xb = X + off, *Rb = Rv + off, *Pb = P + off, *Wb = W + off;
  const double *Qb = Q + off;
  // ---- alpha step -----------------------------------------------------------
  if (mode == 0) {
    const double alpha = active ? rho_a[si] / pq_a[si] : 0.0;
    if (active) {
      for (int R = 0; R < B.nrt; ++R) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * R + 4 * r + q;
          if (row < B.n) {
            const int64_t e = (int64_t)row * N + colj;
            Xb[e] = fma(alpha, Pb[e], Xb[e]);
            Rb[e] = fma(-alpha, Qb[e], Rb[e]);
          }
        }
      }
    }
  }
  // ---- W = T^-T R (backward over column tiles) -----------------------------
  for (int C = B.nrt - 1; C >= 0; --C) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * C + 4 * r + q;
      acc[r] = (row < B.n && colok) ? Rb[(int64_t)row * N + colj] : 0.0;
    }
    const int64_t s0 = ct_ptr[B.rt0 + C], s1 = ct_ptr[B.rt0 + C + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int R = ct_row[t];
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int row = 16 * R + 4 * kc + q;
        const double v = (row < B.n && colok) ? Wb[(int64_t)row * N + colj] : 0.0;
        acc = mfma64(-Tt[(4 * kc + q) * 16 + c], v, acc);
      }
    }
    const double *Ti = tinv + (B.rt0 + C) * 256;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(Ti[(4 * kc + q) * 16 + c], acc[kc], out);
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * C + 4 * r + q;
        if (row < B.n) Wb[(int64_t)row * N + colj] = out[r];
      }
    }
  }
  // ---- W = T^-1 (D W) (forward over row tiles, in place) -------------------
  double rho_new = 0.0;
  for (int R = 0; R < B.nrt; ++R) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * R + 4 * r + q;
      acc[r] = (row < B.n && colok) ? dvec[B.row0 + row] * Wb[(int64_t)row * N + colj] : 0.0;
    }
    const int64_t s0 = rt_ptr[B.rt0 + R], s1 = rt_ptr[B.rt0 + R + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int C = rt_col[t];
      const double *Tt = tiles + (int64_t)rt_slot[t] * 256 + c * 16 + q;
      const double *Wc = Wb + (int64_t)(16 * C + q) * N + coll;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double w = Wc[(int64_t)(4 * kc) * N];
        acc = mfma64(-Tt[4 * kc], colok ? w : 0.0, acc);
      }
    }
    const double *Ti = tinv + (B.rt0 + R) * 256 + c * 16 + q;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(Ti[4 * kc], acc[kc], out);
    if (colok) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * R + 4 * r + q;
        if (row < B.n) {
          const int64_t e = (int64_t)row * N + colj;
          Wb[e] = out[r];
          rho_new = fma(Rb[e], out[r], rho_new);
        }
      }
    }
  }
  rho_new = col_sum(rho_new);
  // ---- direction, convergence ----------------------------------------------
  const double rho_old = colok ? rho_a[si] : 0.0;
  const double rho0 = mode == 1 ? rho_new : (colok ? rho0_a[si] : 0.0);
  const bool now_done = !(rho_new > tol2 * rho0);   // also a zero right-hand side
  const double beta = mode == 0 ? rho_new / rho_old : 0.0;
  if (active) {
    for (int R = 0; R < B.nrt; ++R) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * R + 4 * r + q;
        if (row < B.n) {
          const int64_t e = (int64_t)row * N + colj;
          Pb[e] = mode == 0 ? fma(beta, Pb[e], Wb[e]) : Wb[e];
        }
      }
    }
  }
  if (q == 0 && active) {
    rho_a[si] = rho_new;
    if (mode == 1) rho0_a[si] = rho_new;
    done_a[si] = now_done ? 1.0 : 0.0;
    it_a[si] = mode == 0 ? it_a[si] + 1.0 : (mode == 1 ? 0.0 : it_a[si]);
  }
  const bool going = __any(active && !now_done);
  if (going && lane == 0) atomicAdd(notdone, 1);
}

__global__ void k_pcg_clear(int32_t *notdone) {
  if (threadIdx.x == 0) *notdone = 0;
}

}  // namespace

// Scalars and counter of the iteration inside the workspace.
static double *pcg_scalars(enkfmc_plan *p) { return (double *)(p->ws + p->lay.pcg); }
static int32_t *pcg_counter(enkfmc_plan *p) {
  return (int32_t *)(p->ws + p->lay.pcg + (size_t)kScalars * p->blocks.size() * p->N * sizeof(double));
}

struct PcgArrays {
  double *X, *R, *P, *Q, *W, *hw, *sc;
  int32_t *notdone;
  int ng;
  unsigned grid;
  int64_t nbN;
};

static PcgArrays pcg_arrays(enkfmc_plan *p, const Dev &d) {
  PcgArrays a;
  a.X = d.Z;       // the solution is the local increment, kept for the reverse pass
  a.R = d.W;
  a.P = d.aux1;
  a.Q = d.aux2;
  a.W = d.ubar;    // W = M^-1 R; also D^-1 T P before each Q
  a.hw = d.red;
  a.sc = pcg_scalars(p);
  a.notdone = pcg_counter(p);
  a.ng = (p->N + 15) / 16;
  a.grid = (unsigned)(p->blocks.size() * (size_t)a.ng);
  a.nbN = (int64_t)p->blocks.size() * p->N;
  return a;
}

// Q = A V (W as the scratch for D^-1 T V); with `iterating` the converged
// columns are skipped and P.Q goes to the pq scalars.
static void pcg_apply_A(enkfmc_plan *p, const Dev &d, const PcgArrays &a, const double *V, bool iterating,
                        hipStream_t s) {
  const double *done = iterating ? a.sc + kDone * a.nbN : nullptr;
  hipLaunchKernelGGL(k_pcg_tv, dim3(a.grid), dim3(64), 0, s, d.blocks, a.ng, d.rt_ptr, d.rt_col, d.rt_slot, d.tiles,
                     d.tdiag, d.dvec, V, p->N, done, a.W);
  hipLaunchKernelGGL(k_pcg_ttv, dim3(a.grid), dim3(64), 0, s, d.blocks, a.ng, d.ct_ptr, d.ct_row, d.ct_slot, d.tiles,
                     d.tdiag, a.hw, (const double *)a.W, V, p->N, done, iterating ? a.sc + kPQ * a.nbN : nullptr,
                     a.Q);
}

static void pcg_step(enkfmc_plan *p, const Dev &d, const PcgArrays &a, int mode, double tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_step, dim3(a.grid), dim3(64), 0, s, d.blocks, a.ng, d.rt_ptr, d.rt_col, d.rt_slot,
                     d.ct_ptr, d.ct_row, d.ct_slot, d.tiles, d.tinv, d.dvec, p->N, a.nbN, mode, tol2, a.X, a.R, a.P,
                     (const double *)a.Q, a.W, a.sc, a.notdone);
}

// Residual R = B - neg (neg = A X, or none when X = 0).
template <typename TX>
static void pcg_residual(enkfmc_plan *p, const Dev &d, const PcgArrays &a, const TX *Xb, int64_t ld,
                         const double *Y, const double *r_diag, const double *AX, hipStream_t s) {
  const int64_t tot = p->n_fit * p->N;
  hipLaunchKernelGGL(k_pcg_neg, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, AX, tot, a.R);
  const int64_t nt = p->m_local * p->N;
  if (nt > 0)
    hipLaunchKernelGGL(k_pcg_rhs<TX>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, d.bobs_o, d.bobs_fit,
                       d.fit_glob, Y, Xb, ld, r_diag, p->m_local, p->N, a.R);
}

static hipError_t read_counter(const PcgArrays &a, hipStream_t s, int32_t *out) {
  hipError_t e = hipMemcpyAsync(out, a.notdone, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

// The k_pcg iterations of one graph launch, captured once per plan and
// tolerance (the kernels' arguments are the plan's workspace arrays).
static hipError_t pcg_graph(enkfmc_plan *p, const Dev &d, const PcgArrays &a, double tol2, hipStream_t s) {
  if (p->pcg_exec && p->pcg_graph_tol2 == tol2 && p->pcg_graph_ws == p->ws) return hipSuccess;
  if (p->pcg_exec) {
    (void)hipGraphExecDestroy((hipGraphExec_t)p->pcg_exec);
    p->pcg_exec = nullptr;
  }
  // captured on a stream of the plan's own (the caller's may be the null
  // stream, which cannot be captured); the graph then runs on the caller's
  (void)s;
  hipError_t e;
  if (!p->pcg_cap_stream) {
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    p->pcg_cap_stream = (void *)cs;
  }
  hipStream_t cs = (hipStream_t)p->pcg_cap_stream;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  for (int k = 0; k < kPcgGraphIters; ++k) {
    pcg_apply_A(p, d, a, a.P, true, cs);
    hipLaunchKernelGGL(k_pcg_clear, dim3(1), dim3(64), 0, cs, a.notdone);
    pcg_step(p, d, a, 0, tol2, cs);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess) return e;
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return e;
  p->pcg_exec = (void *)ex;
  p->pcg_graph_tol2 = tol2;
  p->pcg_graph_ws = p->ws;
  return hipSuccess;
}

template <typename TX>
static hipError_t pcg_typed(enkfmc_plan *p, const Dev &d, const TX *Xb, int64_t ld, const double *Y,
                            const double *r_diag, hipStream_t s, int32_t *converged) {
  const PcgArrays a = pcg_arrays(p, d);
  const double tol2 = p->pcg_rtol * p->pcg_rtol;
  const int64_t tot = p->n_fit * p->N;
  *converged = 0;
  p->pcg_iters = 0;
  p->pcg_refinements = 0;
  // observation weights, X = 0, R = B, first preconditioned residual
  hipLaunchKernelGGL(k_pcg_zero, dim3((unsigned)((p->n_fit + 255) / 256)), dim3(256), 0, s, a.hw, p->n_fit);
  if (p->m_local > 0)
    hipLaunchKernelGGL(k_pcg_obs_w, dim3((unsigned)((p->m_local + 255) / 256)), dim3(256), 0, s, d.bobs_o,
                       d.bobs_fit, r_diag, p->m_local, a.hw);
  hipLaunchKernelGGL(k_pcg_zero, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.X, tot);
  pcg_residual(p, d, a, Xb, ld, Y, r_diag, nullptr, s);
  hipLaunchKernelGGL(k_pcg_clear, dim3(1), dim3(64), 0, s, a.notdone);
  pcg_step(p, d, a, 1, tol2, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = pcg_graph(p, d, a, tol2, s);
  if (e != hipSuccess) return e;
  int32_t left = 0;
  e = read_counter(a, s, &left);
  if (e != hipSuccess) return e;
  int it = 0;
  while (true) {
    while (left > 0 && it < p->pcg_maxit) {
      e = hipGraphLaunch((hipGraphExec_t)p->pcg_exec, s);
      if (e != hipSuccess) return e;
      it += kPcgGraphIters;
      e = read_counter(a, s, &left);
      if (e != hipSuccess) return e;
    }
    if (left > 0) break;                       // not converged within maxit
    // FP64 refinement: the true residual of X
    pcg_apply_A(p, d, a, a.X, false, s);
    pcg_residual(p, d, a, Xb, ld, Y, r_diag, a.Q, s);
    hipLaunchKernelGGL(k_pcg_clear, dim3(1), dim3(64), 0, s, a.notdone);
    pcg_step(p, d, a, 2, tol2, s);
    e = read_counter(a, s, &left);
    if (e != hipSuccess) return e;
    if (left == 0) {
      *converged = 1;
      break;
    }
    if (++p->pcg_refinements > kPcgMaxRefinements || it >= p->pcg_maxit) break;
  }
  p->pcg_iters = it;
  return hipGetLastError();
}

hipError_t launch_analysis_pcg(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld,
                               const double *Y, const double *r_diag, hipStream_t s, int32_t *converged) {
  phase_begin(p, ENKFMC_PH_PCG, s);
  hipError_t e = dtype == ENKFMC_F32 ? pcg_typed(p, d, (const float *)Xb, ld, Y, r_diag, s, converged)
                                     : pcg_typed(p, d, (const double *)Xb, ld, Y, r_diag, s, converged);
  phase_end(p, ENKFMC_PH_PCG, s);
  return e;
}

// Largest per-column iteration count and relative residual of the last solve.
hipError_t pcg_column_stats(enkfmc_plan *p, hipStream_t s, int32_t *max_iter, double *max_rel) {
  const size_t nbN = p->blocks.size() * (size_t)p->N;
  std::vector<double> h(kScalars * nbN);
  hipError_t e = hipMemcpyAsync(h.data(), pcg_scalars(p), h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  double mi = 0.0, mr = 0.0;
  for (size_t i = 0; i < nbN; ++i) {
    mi = std::max(mi, h[kIter * nbN + i]);
    const double r0 = h[kRho0 * nbN + i];
    if (r0 > 0.0) mr = std::max(mr, std::sqrt(std::max(0.0, h[kRho * nbN + i]) / r0));
  }
  *max_iter = (int32_t)mi;
  *max_rel = mr;
  return hipSuccess;
}

size_t pcg_scalar_bytes(const enkfmc_plan *p) {
  return (size_t)kScalars * p->blocks.size() * p->N * sizeof(double) + 64;
}

}  // namespace enkfmc
