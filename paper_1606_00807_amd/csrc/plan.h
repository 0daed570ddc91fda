// Internal plan of the EnKF-MC library: host decomposition + device layout.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/enkfmc.h"

namespace enkfmc {

// One (sub-domain, variable) block.  T, D and the local system are
// block-diagonal per variable, so the block is the unit of every solve.
struct Block {
  int32_t sd, var;       // sub-domain, variable
  int32_t nlev, BY, BX;  // local box: levels x latitudes x longitudes
  int32_t n;             // rows = nlev*BY*BX
  int32_t m;             // observations inside the block
  int32_t sd_row0;       // first row of the block in its sub-domain's local order
  int64_t row0;          // first fit row (global fit numbering)
  int64_t nz0;           // first CSR entry of the block
  int64_t obs0;          // first entry of the block's observation list
  int64_t F0;            // offset of the block's F = T^-T H^T (16*nrt x ldf, row-major)
  int64_t S0;            // offset of the block's ldf x ldf innovation matrix
  int64_t Q0;            // offset of the block's ldf x N solve
  int32_t nrt;           // 16-row tiles of the block (the last one may be partial)
  int32_t ldf;           // observation count rounded up to 16
  int64_t rt0;           // first row tile (global row-tile numbering)
  int64_t ot0;           // first observation tile (global numbering; ldf / 16 tiles)
  int32_t far_lo;        // smallest distance R - C beyond the plan's near_d among the block's tiles (0: none)
  int32_t far_w;         // the block's far range: far_lo .. far_lo + far_w - 1 holds its other distances
};

// Buckets of the batched fit: rows grouped by the kernel that fits them.
constexpr int kBucketP0 = 0;      // no predecessors: d = u^T u / (N - 1)
                                  // 1..8: p < N, ceil(p/16) tiles (p-form)
constexpr int kBucketKF = 9;      // p >= N: kernel form, N x N system
constexpr int kBucketPlain = 10;  // beyond the one-wavefront kernels (N > 128, p > 192, or
                                  // 32-bit offsets into U would overflow): the plain kernel
constexpr int kBuckets = 11;
constexpr int kBatchedMaxN = 128;  // largest N of the one-wavefront kernels
constexpr int kBatchedMaxP = 192;  // largest predecessor count of the one-wavefront kernels

struct SubBox {
  int32_t kx, ky, x0, x1, y0, y1, xs, BX, ys, BY, ring;
  int32_t blk0;          // first block of the sub-domain
  int64_t n_sd, nnz_sd, m_sd;
};

// Offsets (bytes) of every device array inside the workspace.
struct Layout {
  size_t blocks, fit_glob, fit_blk, fit_rows, row_ptr, col, csc_ptr, csc_row, csc_nz, interior_src, bobs_o, bobs_row;
  size_t g2f_ptr, g2f, o2b_ptr, o2b, bobs_fit, ot_jmax;
  size_t rt_ptr, rt_col, rt_slot, rt_nfar, ct_ptr, ct_row, ct_slot, ct_nfar, tile_eoff;
  size_t tval, dvec, mean, U, Z, F, S, Q, P, W, aux1, aux2, aux3, dbar, red, tiles, tinv, tdiag, ubar, pcg, status;
  size_t total;
};

}  // namespace enkfmc

struct enkfmc_plan {
  // geometry and sizes
  int32_t nx, ny, nvar, periodic_x, sdx, sdy, r_h, r_v, N;
  std::vector<int32_t> nlev, var_off;
  int64_t n = 0, m = 0;
  int32_t ldu = 0;                 // row stride of the anomaly array (N rounded up to 16)
  std::vector<int32_t> obs_idx;
  // decomposition
  std::vector<enkfmc::SubBox> subs;
  std::vector<enkfmc::Block> blocks;
  std::vector<int32_t> fit_glob, fit_blk;       // per fit row
  std::vector<int32_t> fit_rows;                // fit rows grouped by regression size (see bucket_off)
  int64_t bucket_off[enkfmc::kBuckets + 1] = {};        // rows of bucket b: fit_rows[bucket_off[b], bucket_off[b + 1])
  std::vector<int64_t> row_ptr;                 // n_fit + 1, global CSR offsets
  std::vector<int32_t> col;                     // block-local predecessor rows
  std::vector<int64_t> csc_ptr;                 // n_fit + 1, transposed pattern
  std::vector<int32_t> csc_row, csc_nz;         // block-local row i and entry (relative to nz0) of T_iq
  std::vector<int32_t> interior_src;            // n: fit row that maps back onto each component
  std::vector<int32_t> bobs_o, bobs_row;        // per block observation list
  std::vector<int32_t> bobs_fit;                // fit row of each block observation
  std::vector<int32_t> ot_jmax;                 // per observation tile: largest local row observed in it
  std::vector<int64_t> g2f_ptr;                 // n + 1: fit rows holding each component, sub-domain order
  std::vector<int32_t> g2f;
  std::vector<int64_t> o2b_ptr;                 // m + 1: block-observation entries of each observation
  std::vector<int32_t> o2b;
  // block-sparse 16x16 tiling of T: per row tile the strictly-earlier column
  // tiles holding entries (ascending), per column tile the later row tiles
  std::vector<int64_t> rt_ptr, ct_ptr;          // n_rt + 1
  std::vector<int32_t> rt_col, ct_row;          // tile indices inside the block
  std::vector<int32_t> rt_slot, ct_slot;        // dense tile slot
  std::vector<int32_t> rt_nfar;                 // per row tile: tiles with R - C > near_d (a prefix of its list)
  std::vector<int32_t> ct_nfar;                 // per column tile: tiles with R - C > near_d (a suffix of its list)
  // per row tile rt and row i: at 16 (rt_ptr[rt] + rt + t) + i the offset, in
  // the row's CSR range, of its first entry in tile t of rt's list (t = number
  // of off-diagonal tiles: the diagonal tile); a row's entries are ascending,
  // so those of tile t end where tile t + 1 begins (the diagonal at the row's end)
  std::vector<uint16_t> tile_eoff;
  int64_t n_rt = 0, n_slots = 0;
  int32_t max_rt_tiles = 0;
  int32_t max_rt_back = 0;     // largest R - C over the stored tiles T_RC (C < R) of any block
  int32_t near_d = 0;          // near distance of the split sweeps: the run 1..near_d of R - C values present
  int32_t far_lo = 0;          // smallest R - C value beyond near_d over all blocks (0 if none)
  int32_t far_w = 0;           // widest far range of a block (Block::far_w)
  int64_t n_fit = 0, nnz = 0, m_local = 0, sum_F = 0, sum_S = 0, sum_Q = 0;
  int32_t max_p = 0, max_bn = 0, max_bm = 0;
  enkfmc::Layout lay{};
  // device state
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int32_t device = -1;
  int32_t fitted = 0, analyzed = 0;
  int32_t fit_mode = 0;            // enkfmc_fit_mode of the last fit (the reverse pass uses the same form)
  double fit_ridge = 0.0;
  const void *fit_xb = nullptr;
  const void *an_y = nullptr, *an_r = nullptr;  // Y and r_diag of the last analysis
  // optional per-phase timing with HIP events on the call's stream
  int32_t timing = 0;
  int32_t async = 0;               // calls neither clear nor read the status word (enkfmc_set_async)
  int32_t an_solver = 0;           // enkfmc_solver of the last analysis
  // kernel-form factor cache (enkfmc_plan_set_factor_cache): caller-owned
  // device memory; valid once a batched fit with a ridge has filled it
  double *fcache = nullptr;
  int32_t fcache_valid = 0;
  // preconditioned CG of the local systems (ENKFMC_SOLVE_PCG)
  int32_t pcg_maxit = 2000;
  double pcg_rtol = 1e-12;
  int32_t pcg_iters = 0, pcg_refinements = 0;
  void *pcg_exec = nullptr;        // hipGraphExec_t of a run of iterations
  void *pcg_cap_stream = nullptr;  // stream the graph was captured on
  double pcg_graph_tol2 = -1.0;
  const char *pcg_graph_ws = nullptr;
  void *ev[64] = {};
  uint64_t recorded = 0;
  double phase_ms[32] = {};
};

namespace enkfmc {
// Factor cache (enkfmc_plan_set_factor_cache): a slot of T(T + 1)/2 tiles of
// 256 doubles per row of the one-wavefront buckets 1..8 (p-form, T = b) and
// of the kernel-form bucket (T = ceil(N/16)), bucket after bucket, each in
// the bucket's row order.  fcache_tiles: T of bucket b; fcache_offset:
// doubles before the slots of bucket b (b = kBucketKF + 1: the total).
inline int fcache_tiles(const enkfmc_plan *p, int b) { return b == kBucketKF ? (p->N + 15) / 16 : b; }
inline size_t fcache_offset(const enkfmc_plan *p, int b) {
  size_t off = 0;
  for (int k = 1; k < b && k <= kBucketKF; ++k) {
    const size_t T = (size_t)fcache_tiles(p, k);
    off += (size_t)(p->bucket_off[k + 1] - p->bucket_off[k]) * (T * (T + 1) / 2) * 256;
  }
  return off;
}

enkfmc_status build_plan(enkfmc_plan *p, const enkfmc_geometry *g, int32_t N, const int32_t *obs_idx, int32_t m,
                         std::string *err);
void compute_layout(enkfmc_plan *p);
}  // namespace enkfmc
