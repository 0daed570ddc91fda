// C ABI entry points (include/enkfmc.h).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>

#include "device.h"

using namespace enkfmc;

static thread_local std::string g_err;

static enkfmc_status fail(enkfmc_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

static enkfmc_status hip_fail(hipError_t e, const char *where) {
  return fail(ENKFMC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, where)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// The status word is cleared by a kernel rather than a memset, so that a call
// captured into a HIP graph records no memset node.
__global__ void k_status_clear(int32_t *status) {
  if (threadIdx.x < 16) status[threadIdx.x] = 0;
}

// The device's constant-rate wall clock, written by one thread.
__global__ void k_timestamp(uint64_t *out) {
  if (threadIdx.x == 0) *out = wall_clock64();
}

static hipError_t clear_status(enkfmc_plan *p, hipStream_t s) {
  hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(64), 0, s, (int32_t *)(p->ws + p->lay.status));
  return hipGetLastError();
}

static enkfmc_status decode_status(const int32_t st[2], const char *what) {
  if (st[0] == 0) return ENKFMC_OK;
  std::string where;
  if (st[1] >= 0) where = " (fit row " + std::to_string(st[1]) + ")";
  else where = " (block " + std::to_string(-1 - st[1]) + ")";
  const char *why = st[0] == ENKFMC_ENOTSPD ? "matrix not positive definite"
                    : st[0] == ENKFMC_ENONPOS_D ? "residual variance not positive"
                    : st[0] == ENKFMC_ENOCONV   ? "iteration did not converge"
                                                : "device error";
  return fail((enkfmc_status)st[0], std::string(what) + ": " + why + where);
}

// Read back the device status word (the one device->host read of each call).
// In asynchronous mode the call returns at once: errors stay in the status
// word until enkfmc_check_status reads it.
static enkfmc_status finish(enkfmc_plan *p, hipStream_t s, const char *what) {
  if (p->async) {
    HIPCHK(hipGetLastError(), what);
    return ENKFMC_OK;
  }
  int32_t st[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(st, p->ws + p->lay.status, sizeof(st), hipMemcpyDeviceToHost, s), what);
  HIPCHK(hipStreamSynchronize(s), what);
  if (p->timing) {
    for (int ph = 0; ph < ENKFMC_PH_COUNT; ++ph) {
      if (!(p->recorded & (uint64_t(1) << ph))) continue;
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, (hipEvent_t)p->ev[2 * ph], (hipEvent_t)p->ev[2 * ph + 1]), what);
      p->phase_ms[ph] = ms;
    }
    p->recorded = 0;
  }
  return decode_status(st, what);
}

// Bytes of the factor cache: the factored tiles of every row of the
// one-wavefront buckets (layout in plan.h).
static size_t factor_cache_bytes(const enkfmc_plan *p) { return fcache_offset(p, kBucketKF + 1) * sizeof(double); }

static enkfmc_status begin(enkfmc_plan *p, hipStream_t s, const char *what) {
  if (!p->ws) return fail(ENKFMC_ESTATE, std::string(what) + ": no workspace (call enkfmc_plan_set_workspace)");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev), what);
  if (dev != p->device) return fail(ENKFMC_ESTATE, std::string(what) + ": current device differs from the workspace's");
  if (!p->async) HIPCHK(clear_status(p, s), what);
  if (p->timing) {   // a timed call reports only the phases it runs
    for (double &ms : p->phase_ms) ms = 0.0;
    p->recorded = 0;
  }
  return ENKFMC_OK;
}

template <typename T>
static hipError_t put(enkfmc_plan *p, size_t off, const std::vector<T> &v, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(p->ws + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

extern "C" {

enkfmc_status enkfmc_plan_create(enkfmc_plan **out, const enkfmc_geometry *g, int32_t N, const int32_t *obs_idx,
                                 int32_t m) {
  if (!out) return fail(ENKFMC_EINVAL, "out is NULL");
  *out = nullptr;
  enkfmc_plan *p = new (std::nothrow) enkfmc_plan();
  if (!p) return fail(ENKFMC_ENOMEM, "plan allocation failed");
  std::string err;
  enkfmc_status st;
  try {
    st = build_plan(p, g, N, obs_idx, m, &err);
  } catch (const std::bad_alloc &) {
    st = ENKFMC_ENOMEM;
    err = "host allocation failed while building the plan";
  }
  if (st != ENKFMC_OK) {
    delete p;
    return fail(st, "plan_create: " + err);
  }
  *out = p;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_plan_get_info(const enkfmc_plan *p, enkfmc_plan_info *info) {
  if (!p || !info) return fail(ENKFMC_EINVAL, "plan_get_info: NULL argument");
  info->n = p->n;
  info->N = p->N;
  info->m = p->m;
  info->n_subdomains = (int64_t)p->subs.size();
  info->n_blocks = (int64_t)p->blocks.size();
  info->n_fit = p->n_fit;
  info->nnz = p->nnz;
  info->m_local = p->m_local;
  info->max_p = p->max_p;
  info->max_block_rows = p->max_bn;
  info->max_block_obs = p->max_bm;
  info->reserved = 0;
  info->workspace_bytes = p->lay.total;
  info->fit_rows_plain = p->bucket_off[kBucketPlain + 1] - p->bucket_off[kBucketPlain];
  info->fit_rows_wave = p->n_fit - info->fit_rows_plain;
  info->n_row_tiles = p->n_rt;
  info->n_tiles = p->n_slots;
  info->f_entries = p->sum_F;
  info->s_entries = p->sum_S;
  info->factor_cache_bytes = factor_cache_bytes(p);
  info->near_d = p->near_d;
  info->far_lo = p->far_lo;
  info->max_tile_distance = p->max_rt_back;
  info->far_ring = p->far_w;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_plan_set_factor_cache(enkfmc_plan *p, void *dev, size_t bytes) {
  if (!p) return fail(ENKFMC_EINVAL, "set_factor_cache: NULL plan");
  p->fcache_valid = 0;
  if (!dev) {
    p->fcache = nullptr;
    return ENKFMC_OK;
  }
  if ((reinterpret_cast<uintptr_t>(dev) & 255) != 0)
    return fail(ENKFMC_EINVAL, "set_factor_cache: not 256-byte aligned");
  const size_t need = factor_cache_bytes(p);
  if (bytes < need)
    return fail(ENKFMC_ENOMEM, "set_factor_cache: need " + std::to_string(need) + " bytes, got " +
                                   std::to_string(bytes));
  p->fcache = (double *)dev;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_plan_set_workspace(enkfmc_plan *p, void *dev, size_t bytes, void *stream) {
  if (!p || !dev) return fail(ENKFMC_EINVAL, "set_workspace: NULL argument");
  if ((reinterpret_cast<uintptr_t>(dev) & 255) != 0) return fail(ENKFMC_EINVAL, "set_workspace: not 256-byte aligned");
  if (bytes < p->lay.total)
    return fail(ENKFMC_ENOMEM, "set_workspace: need " + std::to_string(p->lay.total) + " bytes, got " +
                                   std::to_string(bytes));
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipGetDevice(&p->device), "set_workspace");
  p->ws = (char *)dev;
  p->ws_bytes = bytes;
  p->fitted = p->analyzed = 0;
  const Layout &L = p->lay;
  HIPCHK(hipMemcpyAsync(p->ws + L.blocks, p->blocks.data(), p->blocks.size() * sizeof(Block), hipMemcpyHostToDevice, s),
         "set_workspace");
  HIPCHK(put(p, L.fit_glob, p->fit_glob, s), "set_workspace");
  HIPCHK(put(p, L.fit_blk, p->fit_blk, s), "set_workspace");
  HIPCHK(put(p, L.fit_rows, p->fit_rows, s), "set_workspace");
  HIPCHK(put(p, L.row_ptr, p->row_ptr, s), "set_workspace");
  HIPCHK(put(p, L.col, p->col, s), "set_workspace");
  HIPCHK(put(p, L.csc_ptr, p->csc_ptr, s), "set_workspace");
  HIPCHK(put(p, L.csc_row, p->csc_row, s), "set_workspace");
  HIPCHK(put(p, L.csc_nz, p->csc_nz, s), "set_workspace");
  HIPCHK(put(p, L.interior_src, p->interior_src, s), "set_workspace");
  HIPCHK(put(p, L.bobs_o, p->bobs_o, s), "set_workspace");
  HIPCHK(put(p, L.bobs_row, p->bobs_row, s), "set_workspace");
  HIPCHK(put(p, L.g2f_ptr, p->g2f_ptr, s), "set_workspace");
  HIPCHK(put(p, L.g2f, p->g2f, s), "set_workspace");
  HIPCHK(put(p, L.o2b_ptr, p->o2b_ptr, s), "set_workspace");
  HIPCHK(put(p, L.o2b, p->o2b, s), "set_workspace");
  HIPCHK(put(p, L.bobs_fit, p->bobs_fit, s), "set_workspace");
  HIPCHK(put(p, L.ot_jmax, p->ot_jmax, s), "set_workspace");
  HIPCHK(put(p, L.rt_ptr, p->rt_ptr, s), "set_workspace");
  HIPCHK(put(p, L.rt_col, p->rt_col, s), "set_workspace");
  HIPCHK(put(p, L.rt_slot, p->rt_slot, s), "set_workspace");
  HIPCHK(put(p, L.rt_nfar, p->rt_nfar, s), "set_workspace");
  HIPCHK(put(p, L.ct_nfar, p->ct_nfar, s), "set_workspace");
  HIPCHK(put(p, L.ct_ptr, p->ct_ptr, s), "set_workspace");
  HIPCHK(put(p, L.ct_row, p->ct_row, s), "set_workspace");
  HIPCHK(put(p, L.ct_slot, p->ct_slot, s), "set_workspace");
  HIPCHK(put(p, L.tile_eoff, p->tile_eoff, s), "set_workspace");
  // the dense tiles of T hold zeros off the pattern, which no kernel writes
  // (the batched fit writes pattern positions only)
  HIPCHK(hipMemsetAsync(p->ws + L.tiles, 0, (size_t)p->n_slots * 256 * sizeof(double), s), "set_workspace");
  HIPCHK(hipMemsetAsync(p->ws + L.tdiag, 0, (size_t)p->n_rt * 256 * sizeof(double), s), "set_workspace");
  HIPCHK(clear_status(p, s), "set_workspace");
  HIPCHK(hipStreamSynchronize(s), "set_workspace");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_fit(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, double ridge, int32_t mode,
                         void *stream) {
  if (!p || !Xb) return fail(ENKFMC_EINVAL, "fit: NULL argument");
  if (dtype != ENKFMC_F32 && dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "fit: bad dtype");
  if (ld < p->N) return fail(ENKFMC_EINVAL, "fit: ld < N");
  if (!(ridge >= 0.0) || ridge > 1e300) return fail(ENKFMC_EINVAL, "fit: ridge must be finite and >= 0");
  if (mode != ENKFMC_FIT_PLAIN && mode != ENKFMC_FIT_BATCHED && mode != ENKFMC_FIT_SVD)
    return fail(ENKFMC_EINVAL, "fit: bad mode");
  hipStream_t s = (hipStream_t)stream;
  enkfmc_status st = begin(p, s, "fit");
  if (st != ENKFMC_OK) return st;
  p->fitted = p->analyzed = 0;
  p->fcache_valid = 0;
  const Dev d = make_dev(p);
  HIPCHK(launch_anomaly(p, d, Xb, dtype, ld, s), "fit: anomaly launch");
  const bool plain_rows = mode == ENKFMC_FIT_PLAIN ||
                          (mode == ENKFMC_FIT_BATCHED && p->bucket_off[kBucketPlain + 1] > p->bucket_off[kBucketPlain]);
  if (plain_rows && !fit_plain_fits(p))
    return fail(ENKFMC_EUNSUPPORTED, "fit: the plain kernel keeps an N x N Gram in LDS; N too large");
  if (mode == ENKFMC_FIT_SVD && fit_svd_max_lds(p, ridge) > 160 * 1024)
    return fail(ENKFMC_EUNSUPPORTED, "fit: SVD mode keeps each design matrix in LDS; regressions too large");
  if (mode == ENKFMC_FIT_PLAIN) {
    HIPCHK(launch_fit_plain(p, d, ridge, s), "fit: plain launch");
  } else if (mode == ENKFMC_FIT_SVD) {
    HIPCHK(launch_fit_svd(p, d, ridge, s), "fit: svd launch");
  } else {
    HIPCHK(launch_fit_batched(p, d, ridge, s), "fit: batched launch");
  }
  if (mode == ENKFMC_FIT_BATCHED && fit_writes_tiles(p)) {
    HIPCHK(launch_tile_inverse(p, d, s), "fit: tile inverse launch");
  } else {
    HIPCHK(launch_build_tiles(p, d, s), "fit: tile launch");
  }
  st = finish(p, s, "fit");
  if (st != ENKFMC_OK) return st;
  p->fitted = 1;
  p->fcache_valid = mode == ENKFMC_FIT_BATCHED && p->fcache != nullptr;
  p->fit_mode = mode;
  p->fit_ridge = ridge;
  p->fit_xb = Xb;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_analyze(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                             const double *r_diag, void *Xa, int32_t out_dtype, int32_t solver, void *stream) {
  if (!p || !Xb || !Xa || (p->m > 0 && (!Y || !r_diag))) return fail(ENKFMC_EINVAL, "analyze: NULL argument");
  if (dtype != ENKFMC_F32 && dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "analyze: bad dtype");
  if (out_dtype != ENKFMC_F32 && out_dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "analyze: bad out_dtype");
  if (ld < p->N) return fail(ENKFMC_EINVAL, "analyze: ld < N");
  if (solver != ENKFMC_SOLVE_DUAL && solver != ENKFMC_SOLVE_PCG) return fail(ENKFMC_EINVAL, "analyze: unknown solver");
  if (solver == ENKFMC_SOLVE_PCG && p->async)
    return fail(ENKFMC_EINVAL, "analyze: the PCG solver reads its convergence on the host; not in asynchronous mode");
  if (!p->fitted || p->fit_xb != Xb) return fail(ENKFMC_ESTATE, "analyze: needs the preceding fit on the same X_b");
  hipStream_t s = (hipStream_t)stream;
  enkfmc_status st = begin(p, s, "analyze");
  if (st != ENKFMC_OK) return st;
  p->analyzed = 0;
  const Dev d = make_dev(p);
  int32_t converged = 1;
  if (solver == ENKFMC_SOLVE_PCG) {
    HIPCHK(launch_analysis_pcg(p, d, Xb, dtype, ld, Y, r_diag, s, &converged), "analyze: pcg");
    HIPCHK(launch_mapback(p, d, Xb, dtype, ld, Xa, out_dtype, s), "analyze: map back");
  } else {
    HIPCHK(launch_analysis_dual(p, d, Xb, dtype, ld, Y, r_diag, Xa, out_dtype, s), "analyze: launch");
  }
  st = finish(p, s, "analyze");
  if (st != ENKFMC_OK) return st;
  if (!converged)
    return fail(ENKFMC_ENOCONV, "analyze: PCG did not reach rtol within " + std::to_string(p->pcg_maxit) +
                                    " iterations");
  p->an_solver = solver;
  p->analyzed = 1;
  p->an_y = Y;
  p->an_r = r_diag;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_analyze_backward(enkfmc_plan *p, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                                      const double *r_diag, const double *dXa, double *dXb, double *dlogR,
                                      double *dridge, void *stream) {
  if (!p || !Xb || !dXa || !dXb || !dridge || (p->m > 0 && (!Y || !r_diag || !dlogR)))
    return fail(ENKFMC_EINVAL, "analyze_backward: NULL argument");
  if (dtype != ENKFMC_F32 && dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "analyze_backward: bad dtype");
  if (ld < p->N) return fail(ENKFMC_EINVAL, "analyze_backward: ld < N");
  if (!p->fitted || !p->analyzed || p->fit_xb != Xb || p->an_y != (const void *)Y || p->an_r != (const void *)r_diag)
    return fail(ENKFMC_ESTATE, "analyze_backward: needs the preceding fit + analyze on the same inputs");
  if (p->N > 128) return fail(ENKFMC_EUNSUPPORTED, "analyze_backward: N > 128");
  hipStream_t s = (hipStream_t)stream;
  enkfmc_status st = begin(p, s, "analyze_backward");
  if (st != ENKFMC_OK) return st;
  const Dev d = make_dev(p);
  // the reverse pass solves with the dual form: after a PCG analysis its
  // factors (F, S and the Cholesky factor of S) are not there yet
  if (p->an_solver == ENKFMC_SOLVE_PCG) HIPCHK(launch_dual_factor(p, d, r_diag, s), "analyze_backward: dual factors");
  HIPCHK(launch_backward(p, d, Xb, dtype, ld, Y, r_diag, p->fit_ridge, dXa, dXb, dlogR, dridge, s),
         "analyze_backward: launch");
  return finish(p, s, "analyze_backward");
}

enkfmc_status enkfmc_perturb_observations(enkfmc_plan *p, const double *y, const double *r_diag, uint64_t seed,
                                          uint64_t cycle, double *Ys, void *stream) {
  if (!p || (p->m > 0 && (!y || !r_diag || !Ys))) return fail(ENKFMC_EINVAL, "perturb_observations: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  enkfmc_status st = begin(p, s, "perturb_observations");
  if (st != ENKFMC_OK) return st;
  HIPCHK(launch_perturb(y, r_diag, p->m, p->N, seed, cycle, Ys, s), "perturb_observations: launch");
  return finish(p, s, "perturb_observations");
}

enkfmc_status enkfmc_analysis_sq_error(enkfmc_plan *p, const void *Xa, int32_t dtype, int64_t ld,
                                       const double *x_ref, double *err, void *stream) {
  if (!p || !Xa || !x_ref || !err) return fail(ENKFMC_EINVAL, "analysis_sq_error: NULL argument");
  if (dtype != ENKFMC_F32 && dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "analysis_sq_error: bad dtype");
  if (ld < p->N) return fail(ENKFMC_EINVAL, "analysis_sq_error: ld < N");
  hipStream_t s = (hipStream_t)stream;
  enkfmc_status st = begin(p, s, "analysis_sq_error");
  if (st != ENKFMC_OK) return st;
  const Dev d = make_dev(p);
  HIPCHK(launch_sq_error(Xa, dtype, ld, p->n, p->N, x_ref, d.dbar, err, s), "analysis_sq_error: launch");
  return finish(p, s, "analysis_sq_error");
}

enkfmc_status enkfmc_analysis_sq_error_noalloc(int64_t n, int32_t N, const void *Xa, int32_t dtype, int64_t ld,
                                               const double *x_ref, double *err, void *stream) {
  if (!Xa || !x_ref || !err) return fail(ENKFMC_EINVAL, "analysis_sq_error_noalloc: NULL argument");
  if (dtype != ENKFMC_F32 && dtype != ENKFMC_F64) return fail(ENKFMC_EINVAL, "analysis_sq_error_noalloc: bad dtype");
  if (n < 0 || N < 1 || ld < N) return fail(ENKFMC_EINVAL, "analysis_sq_error_noalloc: need n >= 0, N >= 1, ld >= N");
  if (n > ENKFMC_SQ_ERROR_NOALLOC_MAX_N || N > ENKFMC_SQ_ERROR_NOALLOC_MAX_MEMBERS)
    return fail(ENKFMC_EUNSUPPORTED, "analysis_sq_error_noalloc: n = " + std::to_string(n) + ", N = " +
                                         std::to_string(N) + " exceed its limits (n <= " +
                                         std::to_string((long long)ENKFMC_SQ_ERROR_NOALLOC_MAX_N) + ", N <= " +
                                         std::to_string(ENKFMC_SQ_ERROR_NOALLOC_MAX_MEMBERS) + ")");
  double *part = nullptr;
  HIPCHK(sq_error_scratch(&part), "analysis_sq_error_noalloc: scratch lookup");
  HIPCHK(launch_sq_error(Xa, dtype, ld, n, N, x_ref, part, err, (hipStream_t)stream),
         "analysis_sq_error_noalloc: launch");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_rmse(const double *sq_err, int64_t M, double *out, void *stream) {
  if (!sq_err || !out || M < 1) return fail(ENKFMC_EINVAL, "rmse: need M >= 1 squared errors and an output");
  HIPCHK(launch_rmse(sq_err, M, out, (hipStream_t)stream), "rmse: launch");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_pattern_sizes(const enkfmc_plan *p, int32_t k, int64_t *n_sd, int64_t *nnz_sd,
                                       int64_t *m_sd) {
  if (!p || k < 0 || k >= (int32_t)p->subs.size()) return fail(ENKFMC_EINVAL, "get_pattern_sizes: bad sub-domain");
  const SubBox &sb = p->subs[k];
  int64_t ms = 0;
  for (int32_t v = 0; v < p->nvar; ++v) ms += p->blocks[sb.blk0 + v].m;
  if (n_sd) *n_sd = sb.n_sd;
  if (nnz_sd) *nnz_sd = sb.nnz_sd;
  if (m_sd) *m_sd = ms;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_pattern(const enkfmc_plan *p, int32_t k, int64_t *loc2glob, uint8_t *interior,
                                 int64_t *row_ptr, int32_t *col_idx, int32_t *obs, int32_t *obs_row) {
  if (!p || k < 0 || k >= (int32_t)p->subs.size()) return fail(ENKFMC_EINVAL, "get_pattern: bad sub-domain");
  const SubBox &sb = p->subs[k];
  const Block &B0 = p->blocks[sb.blk0];
  int64_t nzo = 0, mo = 0;
  if (row_ptr) row_ptr[0] = 0;
  for (int32_t v = 0; v < p->nvar; ++v) {
    const Block &B = p->blocks[sb.blk0 + v];
    for (int32_t i = 0; i < B.n; ++i) {
      const int64_t r = B.row0 + i;
      const int64_t li = B.sd_row0 + i;
      if (loc2glob) loc2glob[li] = p->fit_glob[r];
      if (interior) interior[li] = (uint8_t)(p->interior_src[p->fit_glob[r]] == r);
      for (int64_t t = p->row_ptr[r]; t < p->row_ptr[r + 1]; ++t) {
        if (col_idx) col_idx[nzo] = B.sd_row0 + p->col[t];
        ++nzo;
      }
      if (row_ptr) row_ptr[li + 1] = nzo;
    }
    for (int32_t a = 0; a < B.m; ++a) {
      if (obs) obs[mo] = p->bobs_o[B.obs0 + a];
      if (obs_row) obs_row[mo] = B.sd_row0 + p->bobs_row[B.obs0 + a];
      ++mo;
    }
  }
  (void)B0;
  // observations of a sub-domain are listed variable by variable above; the
  // export orders them by observation number like the paper's local H.
  if (obs && obs_row && mo > 1) {
    std::vector<std::pair<int32_t, int32_t>> t(mo);
    for (int64_t a = 0; a < mo; ++a) t[a] = {obs[a], obs_row[a]};
    std::sort(t.begin(), t.end());
    for (int64_t a = 0; a < mo; ++a) { obs[a] = t[a].first; obs_row[a] = t[a].second; }
  }
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_factors(enkfmc_plan *p, int32_t k, double *tval, double *d, void *stream) {
  if (!p || k < 0 || k >= (int32_t)p->subs.size()) return fail(ENKFMC_EINVAL, "get_factors: bad sub-domain");
  if (!p->fitted) return fail(ENKFMC_ESTATE, "get_factors: no fit yet");
  hipStream_t s = (hipStream_t)stream;
  const SubBox &sb = p->subs[k];
  const Block &B0 = p->blocks[sb.blk0];
  const Dev dv = make_dev(p);
  if (tval && sb.nnz_sd > 0)
    HIPCHK(hipMemcpyAsync(tval, dv.tval + B0.nz0, sb.nnz_sd * 8, hipMemcpyDeviceToHost, s), "get_factors");
  if (d) HIPCHK(hipMemcpyAsync(d, dv.dvec + B0.row0, sb.n_sd * 8, hipMemcpyDeviceToHost, s), "get_factors");
  HIPCHK(hipStreamSynchronize(s), "get_factors");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_increment(enkfmc_plan *p, int32_t k, double *Z, void *stream) {
  if (!p || !Z || k < 0 || k >= (int32_t)p->subs.size()) return fail(ENKFMC_EINVAL, "get_increment: bad argument");
  if (!p->analyzed) return fail(ENKFMC_ESTATE, "get_increment: no analysis yet");
  hipStream_t s = (hipStream_t)stream;
  const SubBox &sb = p->subs[k];
  const Block &B0 = p->blocks[sb.blk0];
  const Dev dv = make_dev(p);
  HIPCHK(hipMemcpyAsync(Z, dv.Z + B0.row0 * p->N, sb.n_sd * p->N * 8, hipMemcpyDeviceToHost, s), "get_increment");
  HIPCHK(hipStreamSynchronize(s), "get_increment");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_set_pcg(enkfmc_plan *p, int32_t maxit, double rtol) {
  if (!p || maxit < 1 || !(rtol > 0.0 && rtol < 1.0)) return fail(ENKFMC_EINVAL, "set_pcg: need maxit >= 1, 0 < rtol < 1");
  p->pcg_maxit = maxit;
  p->pcg_rtol = rtol;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_pcg_stats(enkfmc_plan *p, int32_t *iterations, int32_t *max_column_iterations,
                                   int32_t *refinements, double *max_rel_residual, void *stream) {
  if (!p || !iterations || !max_column_iterations || !refinements || !max_rel_residual)
    return fail(ENKFMC_EINVAL, "get_pcg_stats: NULL argument");
  if (!p->ws) return fail(ENKFMC_ESTATE, "get_pcg_stats: no workspace");
  *iterations = p->pcg_iters;
  *refinements = p->pcg_refinements;
  HIPCHK(pcg_column_stats(p, (hipStream_t)stream, max_column_iterations, max_rel_residual), "get_pcg_stats");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_set_async(enkfmc_plan *p, int32_t enable) {
  if (!p) return fail(ENKFMC_EINVAL, "set_async: NULL plan");
  p->async = enable ? 1 : 0;
  if (p->async) p->timing = 0;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_check_status(enkfmc_plan *p, void *stream) {
  if (!p) return fail(ENKFMC_EINVAL, "check_status: NULL plan");
  if (!p->ws) return fail(ENKFMC_ESTATE, "check_status: no workspace");
  hipStream_t s = (hipStream_t)stream;
  int32_t st[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(st, p->ws + p->lay.status, sizeof(st), hipMemcpyDeviceToHost, s), "check_status");
  HIPCHK(hipStreamSynchronize(s), "check_status");
  if (st[0] != 0) HIPCHK(clear_status(p, s), "check_status");
  return decode_status(st, "check_status");
}

enkfmc_status enkfmc_timestamp(uint64_t *dev, void *stream) {
  if (!dev) return fail(ENKFMC_EINVAL, "timestamp: NULL argument");
  hipLaunchKernelGGL(k_timestamp, dim3(1), dim3(64), 0, (hipStream_t)stream, dev);
  HIPCHK(hipGetLastError(), "timestamp");
  return ENKFMC_OK;
}

enkfmc_status enkfmc_wall_clock_hz(int64_t *hz) {
  if (!hz) return fail(ENKFMC_EINVAL, "wall_clock_hz: NULL argument");
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev), "wall_clock_hz");
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall_clock_hz");
  *hz = (int64_t)khz * 1000;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_set_timing(enkfmc_plan *p, int32_t enable) {
  if (!p) return fail(ENKFMC_EINVAL, "set_timing: NULL plan");
  if (enable && p->async) return fail(ENKFMC_EINVAL, "set_timing: phase timing needs synchronous calls");
  if (enable && !p->ev[0]) {
    for (int i = 0; i < 2 * ENKFMC_PH_COUNT; ++i) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e), "set_timing");
      p->ev[i] = (void *)e;
    }
  }
  p->timing = enable ? 1 : 0;
  p->recorded = 0;
  return ENKFMC_OK;
}

enkfmc_status enkfmc_get_timing(const enkfmc_plan *p, int32_t phase, double *ms) {
  if (!p || !ms || phase < 0 || phase >= ENKFMC_PH_COUNT) return fail(ENKFMC_EINVAL, "get_timing: bad argument");
  *ms = p->phase_ms[phase];
  return ENKFMC_OK;
}

const char *enkfmc_status_string(int32_t st) {
  switch (st) {
    case ENKFMC_OK: return "ENKFMC_OK";
    case ENKFMC_EINVAL: return "ENKFMC_EINVAL";
    case ENKFMC_ENOTSPD: return "ENKFMC_ENOTSPD";
    case ENKFMC_ENONPOS_D: return "ENKFMC_ENONPOS_D";
    case ENKFMC_ENOCONV: return "ENKFMC_ENOCONV";
    case ENKFMC_EHIP: return "ENKFMC_EHIP";
    case ENKFMC_ENOMEM: return "ENKFMC_ENOMEM";
    case ENKFMC_ESTATE: return "ENKFMC_ESTATE";
    case ENKFMC_EUNSUPPORTED: return "ENKFMC_EUNSUPPORTED";
    default: return "ENKFMC_UNKNOWN";
  }
}

const char *enkfmc_last_error(void) { return g_err.c_str(); }

void enkfmc_plan_destroy(enkfmc_plan *p) {
  if (!p) return;
  for (int i = 0; i < 64; ++i)
    if (p->ev[i]) hipEventDestroy((hipEvent_t)p->ev[i]);
  if (p->pcg_exec) hipGraphExecDestroy((hipGraphExec_t)p->pcg_exec);
  if (p->pcg_cap_stream) hipStreamDestroy((hipStream_t)p->pcg_cap_stream);
  delete p;
}

}  // extern "C"
