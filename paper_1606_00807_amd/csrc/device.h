// Device-side view of the workspace and small helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace enkfmc {

struct Dev {
  const Block *blocks;
  const int32_t *fit_glob, *fit_blk, *fit_rows;
  const int64_t *row_ptr;
  const int32_t *col;
  const int64_t *csc_ptr;
  const int32_t *csc_row, *csc_nz;
  const int32_t *interior_src, *bobs_o, *bobs_row;
  const int64_t *g2f_ptr;
  const int32_t *g2f;
  const int64_t *o2b_ptr;
  const int32_t *o2b, *bobs_fit, *ot_jmax;
  const int64_t *rt_ptr, *ct_ptr;
  const int32_t *rt_col, *rt_slot, *rt_nfar, *ct_row, *ct_slot, *ct_nfar;
  const uint16_t *tile_eoff;
  double *tiles, *tinv, *tdiag, *ubar;
  double *tval, *dvec, *mean, *U, *Z, *F, *S, *Q, *P, *W, *aux1, *aux2, *aux3, *dbar, *red;
  int32_t *status;
};

inline Dev make_dev(enkfmc_plan *p) {
  char *w = p->ws;
  const Layout &L = p->lay;
  Dev d;
  d.blocks = (const Block *)(w + L.blocks);
  d.fit_glob = (const int32_t *)(w + L.fit_glob);
  d.fit_blk = (const int32_t *)(w + L.fit_blk);
  d.fit_rows = (const int32_t *)(w + L.fit_rows);
  d.row_ptr = (const int64_t *)(w + L.row_ptr);
  d.col = (const int32_t *)(w + L.col);
  d.csc_ptr = (const int64_t *)(w + L.csc_ptr);
  d.csc_row = (const int32_t *)(w + L.csc_row);
  d.csc_nz = (const int32_t *)(w + L.csc_nz);
  d.interior_src = (const int32_t *)(w + L.interior_src);
  d.bobs_o = (const int32_t *)(w + L.bobs_o);
  d.bobs_row = (const int32_t *)(w + L.bobs_row);
  d.g2f_ptr = (const int64_t *)(w + L.g2f_ptr);
  d.g2f = (const int32_t *)(w + L.g2f);
  d.o2b_ptr = (const int64_t *)(w + L.o2b_ptr);
  d.o2b = (const int32_t *)(w + L.o2b);
  d.bobs_fit = (const int32_t *)(w + L.bobs_fit);
  d.ot_jmax = (const int32_t *)(w + L.ot_jmax);
  d.rt_ptr = (const int64_t *)(w + L.rt_ptr);
  d.rt_col = (const int32_t *)(w + L.rt_col);
  d.rt_slot = (const int32_t *)(w + L.rt_slot);
  d.rt_nfar = (const int32_t *)(w + L.rt_nfar);
  d.ct_nfar = (const int32_t *)(w + L.ct_nfar);
  d.ct_ptr = (const int64_t *)(w + L.ct_ptr);
  d.ct_row = (const int32_t *)(w + L.ct_row);
  d.ct_slot = (const int32_t *)(w + L.ct_slot);
  d.tile_eoff = (const uint16_t *)(w + L.tile_eoff);
  d.tiles = (double *)(w + L.tiles);
  d.tinv = (double *)(w + L.tinv);
  d.tdiag = (double *)(w + L.tdiag);
  d.ubar = (double *)(w + L.ubar);
  d.tval = (double *)(w + L.tval);
  d.dvec = (double *)(w + L.dvec);
  d.mean = (double *)(w + L.mean);
  d.U = (double *)(w + L.U);
  d.Z = (double *)(w + L.Z);
  d.F = (double *)(w + L.F);
  d.S = (double *)(w + L.S);
  d.Q = (double *)(w + L.Q);
  d.P = (double *)(w + L.P);
  d.W = (double *)(w + L.W);
  d.aux1 = (double *)(w + L.aux1);
  d.aux2 = (double *)(w + L.aux2);
  d.aux3 = (double *)(w + L.aux3);
  d.dbar = (double *)(w + L.dbar);
  d.red = (double *)(w + L.red);
  d.status = (int32_t *)(w + L.status);
  return d;
}

// A v_mfma_f64_16x16x4 accumulator (four doubles per lane).  Lane l = 16q + c
// holds element (4r + q, c) in register r; the A operand of a product is
// A[c][q] at lane (q, c), the B operand B[q][c].
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ inline d4 mfma64(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

// Orders one wavefront's LDS accesses where lanes exchange values through
// LDS: a wavefront executes its LDS instructions in issue order, so a read
// issued after a write sees it; this only keeps the compiler from moving
// memory operations across this point.
__device__ inline void wave_lds_sync() {
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Row Q of the wavefront (lanes 16Q..16Q+15), given to all four rows, lane
// 16q + c receiving lane 16Q + c.  With rows written (r0, r1, r2, r3): the
// 16-lane swap of the low and high words (lo, hi) leaves (lo0, hi0, lo2, hi2)
// in its first result and (lo1, hi1, lo3, hi3) in its second; the 32-lane swap
// of one of them with itself leaves (loQ, hiQ, loQ, hiQ) in one result; the
// 16-lane swap of that with itself leaves loQ in all rows of its first result
// and hiQ in all rows of its second.
template <int Q>
__device__ __forceinline__ double quarter_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const auto s1 = __builtin_amdgcn_permlane16_swap((unsigned)(b & 0xffffffffll), (unsigned)(b >> 32), false, false);
  const unsigned t = (Q & 1) ? s1[1] : s1[0];
  const auto s2 = __builtin_amdgcn_permlane32_swap(t, t, false, false);
  const unsigned u = (Q & 2) ? s2[1] : s2[0];
  const auto s3 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  return __longlong_as_double(((long long)s3[1] << 32) | s3[0]);
}

// First error wins; status[1] records where it happened.
// MI355X dispatches the workgroups of a launch to its 8 XCDs in turn
// (workgroup b to XCD b mod 8), and each XCD has an L2 of its own.  This maps
// b to a logical index such that every XCD runs one contiguous range of
// logical workgroups (a bijection on [0, G)): neighbouring rows, which share
// most of their predecessors' rows of U, then meet in the same L2.
constexpr int kXcds = 8;

// Largest ring of 16x16 tiles a triangular sweep keeps in LDS (one
// workgroup's dynamic LDS); plans that need more use the sweeps without one.
constexpr size_t kRingMaxBytes = 64 * 1024;
// Largest gap ring (the near run and a block's far range of tiles) of the
// triangular sweeps.
constexpr size_t kGapRingMaxBytes = 32 * 1024;
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t G) {
  const int64_t x = b % kXcds, s = b / kXcds, q = G / kXcds, rm = G % kXcds;
  return x < rm ? x * (q + 1) + s : rm * (q + 1) + (x - rm) * q + s;
}

// Decode of a one-dimensional launch over (block, tile) pairs, logical index
// block * per_block + tile, numbered XCD-contiguously: the tiles of one block
// are neighbouring workgroups on one XCD and share the block's data in its L2.
__device__ __forceinline__ void block_tile(int per_block, int &blk, int &tile) {
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  blk = (int)(lg / per_block);
  tile = (int)(lg % per_block);
}

__device__ inline void set_error(int32_t *status, int32_t code, int32_t where) {
  if (atomicCAS(status, 0, code) == 0) atomicExch(status + 1, where);
}

// Sum over a 64-lane wavefront; every lane gets the same, order-fixed result.
__device__ inline double wave_sum(double s) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// Sum over a 256-thread workgroup (red: >= 4 doubles of LDS).  Order-fixed.
__device__ inline double block_sum256(double s, double *red) {
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

template <typename T> __device__ inline double ld_as_double(const T *p) { return (double)(*p); }

// In-place solve L L^T x = x for one column x (stride sx) with the lower
// Cholesky factor L (m x m, row stride ld), eight rows at a time: each loaded
// x_b serves eight independent accumulations.
__device__ inline void chol_solve_col(const double *__restrict__ L, int ld, int m, double *__restrict__ x,
                                      int64_t sx) {
  constexpr int kB = 8;
  for (int a0 = 0; a0 < m; a0 += kB) {          // forward: L y = x
    double acc[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) acc[i] = a0 + i < m ? x[(int64_t)(a0 + i) * sx] : 0.0;
    for (int b = 0; b < a0; ++b) {
      const double xb = x[(int64_t)b * sx];
#pragma unroll
      for (int i = 0; i < kB; ++i)
        if (a0 + i < m) acc[i] = fma(-L[(int64_t)(a0 + i) * ld + b], xb, acc[i]);
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {
      const int a = a0 + i;
      if (a < m) {
#pragma unroll
        for (int j = 0; j < i; ++j) acc[i] = fma(-L[(int64_t)a * ld + a0 + j], acc[j], acc[i]);
        acc[i] /= L[(int64_t)a * ld + a];
        x[(int64_t)a * sx] = acc[i];
      }
    }
  }
  const int top = (m - 1) / kB * kB;
  for (int a0 = top; a0 >= 0; a0 -= kB) {       // backward: L^T x = y
    double acc[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) acc[i] = a0 + i < m ? x[(int64_t)(a0 + i) * sx] : 0.0;
    for (int b = a0 + kB; b < m; ++b) {
      const double xb = x[(int64_t)b * sx];
#pragma unroll
      for (int i = 0; i < kB; ++i) acc[i] = fma(-L[(int64_t)b * ld + a0 + i], xb, acc[i]);
    }
#pragma unroll
    for (int i = kB - 1; i >= 0; --i) {
      const int a = a0 + i;
      if (a < m) {
#pragma unroll
        for (int j = i + 1; j < kB; ++j)
          if (a0 + j < m) acc[i] = fma(-L[(int64_t)(a0 + j) * ld + a], acc[j], acc[i]);
        acc[i] /= L[(int64_t)a * ld + a];
        x[(int64_t)a * sx] = acc[i];
      }
    }
  }
}

// Phase timing: records a HIP event pair around a kernel when the plan asks for it.
inline void phase_begin(enkfmc_plan *p, int ph, hipStream_t s) {
  if (!p->timing) return;
  (void)hipEventRecord((hipEvent_t)p->ev[2 * ph], s);
}
inline void phase_end(enkfmc_plan *p, int ph, hipStream_t s) {
  if (!p->timing) return;
  (void)hipEventRecord((hipEvent_t)p->ev[2 * ph + 1], s);
  p->recorded |= (uint64_t(1) << ph);
}

// Host-side launchers (defined in the .hip files).
hipError_t launch_anomaly(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, hipStream_t s);
hipError_t launch_fit_plain(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s);
hipError_t launch_fit_plain_rows(enkfmc_plan *p, const Dev &d, double lam, const int32_t *rows, int64_t nrows,
                                 hipStream_t s);
bool fit_plain_fits(const enkfmc_plan *p);   // the plain kernel's N x N Gram fits in LDS
hipError_t launch_adj_regress_plain_rows(enkfmc_plan *p, const Dev &d, double lam, const int32_t *rows,
                                         int64_t nrows, hipStream_t s);
hipError_t launch_fit_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s);
hipError_t launch_fit_svd(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s);
size_t fit_svd_max_lds(const enkfmc_plan *p, double lam);   // LDS of the largest SVD regression
hipError_t launch_build_tiles(enkfmc_plan *p, const Dev &d, hipStream_t s);
bool fit_writes_tiles(const enkfmc_plan *p);   // the batched fit writes the dense tiles of T itself
hipError_t launch_tile_inverse(enkfmc_plan *p, const Dev &d, hipStream_t s);   // tinv from tdiag
int max_block_tiles(const enkfmc_plan *p);
hipError_t launch_fwd_sweep(enkfmc_plan *p, const Dev &d, const double *Q, const double *V, double *out,
                            hipStream_t s);
hipError_t launch_analysis_pcg(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld,
                               const double *Y, const double *r_diag, hipStream_t s, int32_t *converged);
hipError_t pcg_column_stats(enkfmc_plan *p, hipStream_t s, int32_t *max_iter, double *max_rel);
hipError_t launch_dual_factor(enkfmc_plan *p, const Dev &d, const double *r_diag, hipStream_t s);
// P <- S^-1 P by 16-row tiles with the factor the analysis left in S, for
// plans whose blocks hold at most 128 observations (solve_S_tiles_fit)
bool solve_S_tiles_fit(const enkfmc_plan *p);
// Cholesky of every block's S by 16 x 16 register tiles, one wavefront per
// block, for plans whose blocks hold at most 128 observations
bool dual_chol_tiles_fit(const enkfmc_plan *p);
hipError_t launch_dual_chol_tiles(enkfmc_plan *p, const Dev &d, hipStream_t s);
hipError_t launch_adj_solve_S_tiles(enkfmc_plan *p, const Dev &d, double *P, hipStream_t s);
hipError_t launch_mapback(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, void *Xa,
                          int32_t out_dtype, hipStream_t s);
hipError_t launch_analysis_dual(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld,
                                const double *Y, const double *r_diag, void *Xa, int32_t out_dtype, hipStream_t s);
hipError_t launch_adj_regress_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s);
hipError_t launch_backward(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                           const double *r_diag, double lam, const double *dXa, double *dXb, double *dlogR,
                           double *dridge, hipStream_t s);
hipError_t launch_perturb(const double *y, const double *r_diag, int64_t m, int N, uint64_t seed, uint64_t cycle,
                          double *Ys, hipStream_t s);
// Workgroups of the first level of the squared-error reduction; its partials
// need that many doubles of scratch.
constexpr int kSqErrorParts = 256;
hipError_t launch_sq_error(const void *Xa, int32_t dtype, int64_t ld, int64_t n, int N, const double *xref,
                           double *part, double *out, hipStream_t s);
hipError_t launch_rmse(const double *sq, int64_t M, double *out, hipStream_t s);
// Device address of the current GPU's static scratch for those partials
// (kSqErrorParts doubles), looked up once per device.
hipError_t sq_error_scratch(double **out);

}  // namespace enkfmc
