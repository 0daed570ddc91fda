// Local analysis of every (sub-domain, variable) block and the merge.
//
// The local primal system of eq. (11) (per sub-domain, eq. 14 / Alg. 3),
//   (T^T D^-1 T + H^T R^-1 H) Z = H^T R^-1 Delta,   Delta = Y^s - H X_b,
// is solved exactly through the dual form of eqs. (12)-(13):
//   B^ = T^-1 D T^-T,   F = T^-T H^T            (n_b x m_b, backward sweep)
//   S  = R + H B^ H^T = R + F^T D F             (m_b x m_b, Cholesky)
//   Q  = S^-1 Delta                             (m_b x N)
//   Z  = B^ H^T Q = T^-1 (D (F Q))              (forward sweep, N columns)
// Then X_a = X_b + Z on interior rows only (Alg. 2 merge; the interiors of
// the sub-domains do not intersect, so every component is written once).
//
// Sweeps work on a block-sparse 16x16 tiling of T: rows are cut into 16-row
// tiles (one latitude line of a 16-wide box); row tile R couples to the few
// earlier column tiles holding its predecessors (dense tiles T_RC) and to
// itself (unit lower triangular T_RR, inverted once after the fit).  A sweep
// is then a sequence of v_mfma_f64_16x16x4 tile products per row tile.
//
// v_mfma_f64_16x16x4 conventions (lane l = 16q + c): A operand A[c][q],
// B operand B[q][c], accumulator register r holds element (4r + q, c).
#include <algorithm>

#include "device.h"

namespace enkfmc {


// Dense tiles T_RC (row-major) of row tile R, and the inverse of T_RR.
// One wavefront per (block, row tile).  The CSR entries of the tile's 16 rows
// are contiguous; the wavefront reads them in coalesced runs of 64 and
// scatters each into its tile, assembled in LDS (zeros elsewhere) up to
// kTileChunk tiles at a time, then writes the tiles out whole.  An entry's row
// is found among the 17 row starts (uniform registers), its tile's place in
// the row tile's list through a small LDS map indexed by R - C.  The diagonal
// tile stays in LDS, where 16 lanes invert it.
constexpr int kTileChunk = 13;
constexpr int kTileMap = 128;
constexpr int kBuildUnroll = 8;

__global__ __launch_bounds__(64) void k_build_tiles(const Block *__restrict__ blocks,
                                                    const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ tval,
                                                    const int64_t *__restrict__ rt_ptr,
                                                    const int32_t *__restrict__ rt_col,
                                                    const int32_t *__restrict__ rt_slot, double *__restrict__ tiles,
                                                    double *__restrict__ tinv, double *__restrict__ tdiag) {
  __shared__ double tb[kTileChunk * 256];
  __shared__ double diag[256];
  __shared__ int32_t tmap[kTileMap];
  const Block B = blocks[blockIdx.x];
  const int R = blockIdx.y;
  if (R >= B.nrt) return;
  const int lane = threadIdx.x;
  const int64_t rt = B.rt0 + R;
  const int64_t t0 = rt_ptr[rt];
  const int nt = (int)(rt_ptr[rt + 1] - t0);
  const int nrow = B.n - 16 * R < 16 ? B.n - 16 * R : 16;
  // row starts 0..nrow (the entries of row i are [rs_i, rs_{i+1}))
  const int64_t myrs = lane <= nrow ? row_ptr[B.row0 + 16 * R + lane] : 0;
  int64_t rs[17];
#pragma unroll
  for (int i = 0; i <= 16; ++i) {
    const long long v = __shfl((long long)myrs, i <= nrow ? i : nrow, 64);
    rs[i] = (int64_t)v;
  }
  const int64_t k0 = rs[0], k1 = rs[16];
  for (int t = lane; t < nt; t += 64) {
    const int d = R - rt_col[t0 + t];
    if (d < kTileMap) tmap[d] = t;
  }
  for (int tlo = 0; tlo == 0 || tlo < nt; tlo += kTileChunk) {
    const int thi = nt - tlo < kTileChunk ? nt : tlo + kTileChunk;
    for (int e = lane; e < (thi - tlo) * 256; e += 64) tb[e] = 0.0;
    if (tlo == 0)
      for (int e = lane; e < 256; e += 64) diag[e] = 0.0;
    wave_lds_sync();
    // kBuildUnroll runs of 64 entries are loaded before any is scattered
    for (int64_t kb = k0; kb < k1; kb += 64 * kBuildUnroll) {
      int cs[kBuildUnroll];
      double vs[kBuildUnroll];
#pragma unroll
      for (int u = 0; u < kBuildUnroll; ++u) {
        const int64_t k = kb + 64 * u + lane;
        cs[u] = k < k1 ? col[k] : 0;
        vs[u] = k < k1 ? tval[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kBuildUnroll; ++u) {
        const int64_t k = kb + 64 * u + lane;
        if (k >= k1) continue;
        int i = 0;
#pragma unroll
        for (int h = 1; h < 16; ++h) i += k >= rs[h] ? 1 : 0;
        const int C = cs[u] >> 4, j = cs[u] & 15;
        if (C == R) {
          if (tlo == 0) diag[i * 16 + j] = vs[u];
        } else {
          int t;
          if (R - C < kTileMap) {
            t = tmap[R - C];
          } else {   // list position by bisection (rt_col ascending)
            int lo = 0, hi = nt - 1;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (rt_col[t0 + mid] < C) lo = mid + 1; else hi = mid;
            }
            t = lo;
          }
          if (t >= tlo && t < thi) tb[(t - tlo) * 256 + i * 16 + j] = vs[u];
        }
      }
    }
    wave_lds_sync();
    for (int e = lane; e < (thi - tlo) * 128; e += 64) {
      const int tt = e >> 7, w = 2 * (e & 127);
      *(d2 *)(tiles + (int64_t)rt_slot[t0 + tlo + tt] * 256 + w) = d2{tb[tt * 256 + w], tb[tt * 256 + w + 1]};
    }
    wave_lds_sync();
  }
  for (int e = lane; e < 256; e += 64) tdiag[rt * 256 + e] = diag[e];   // strictly lower T_RR
  if (lane < 16) {
    // column `lane` of (I + L)^-1 by forward substitution
    const int j = lane;
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) v -= diag[i * 16 + k] * x[k];
      x[i] = (i < j) ? 0.0 : v;
    }
    double *dst = tinv + rt * 256;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[i * 16 + j] = x[i];
  }
}

// F = T^-T H^T, backward over row tiles; one wavefront per (block, 16 observation columns).
// T^-T is upper triangular, so the 16 columns vanish below their largest
// observed row: those tiles are only zero-filled and the sweep starts above.
__global__ __launch_bounds__(64) void k_bwd_sweep(const Block *__restrict__ blocks, const int64_t *__restrict__ ct_ptr,
                                                  const int32_t *__restrict__ ct_row,
                                                  const int32_t *__restrict__ ct_slot,
                                                  const int32_t *__restrict__ bobs_row,
                                                  const int32_t *__restrict__ ot_jmax,
                                                  const double *__restrict__ tiles, const double *__restrict__ tinv,
                                                  double *__restrict__ F) {
  const Block B = blocks[blockIdx.x];
  const int oc = blockIdx.y;
  if (16 * oc >= B.m) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int o = 16 * oc + c;
  const int jo = o < B.m ? bobs_row[B.obs0 + o] : -1;
  const int ldf = B.ldf;
  double *Fb = F + B.F0;
  const int Cs = ot_jmax[B.ot0 + oc] >> 4;
  for (int C = B.nrt - 1; C > Cs; --C) {
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) Fc[(int64_t)(4 * r + q) * ldf] = 0.0;
  }
  for (int C = Cs; C >= 0; --C) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = (16 * C + 4 * r + q == jo) ? 1.0 : 0.0;
    // later row tiles R > Cs hold zeros of F; ascending, so they end the list.
    // The loads of tile t + 1 are issued before the MFMAs of tile t.
    const int64_t s0 = ct_ptr[B.rt0 + C];
    int64_t s1 = ct_ptr[B.rt0 + C + 1];
    while (s1 > s0 && ct_row[s1 - 1] > Cs) --s1;
    double ta[4], fa[4];
    auto load = [&](int64_t t, double (&tv)[4], double (&fv)[4]) {
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256;
      const double *Fr = Fb + (int64_t)(16 * ct_row[t]) * ldf + 16 * oc + c;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        tv[kc] = Tt[(4 * kc + q) * 16 + c];
        fv[kc] = Fr[(int64_t)(4 * kc + q) * ldf];
      }
    };
    if (s0 < s1) load(s0, ta, fa);
    for (int64_t t = s0; t < s1; ++t) {
      double tb[4] = {0.0, 0.0, 0.0, 0.0}, fb[4] = {0.0, 0.0, 0.0, 0.0};
      if (t + 1 < s1) load(t + 1, tb, fb);
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc = mfma64(-ta[kc], fa[kc], acc);
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        ta[kc] = tb[kc];
        fa[kc] = fb[kc];
      }
    }
    const double *Ti = tinv + (B.rt0 + C) * 256;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(Ti[(4 * kc + q) * 16 + c], acc[kc], out);
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) Fc[(int64_t)(4 * r + q) * ldf] = out[r];
  }
}

// The same backward sweep with this wavefront's F tiles of the last W column
// tiles done (rows C+1 .. C+W) in an LDS ring, slot R mod W, so T_RC^T F_R reads
// F_R from LDS (every stored T_RC has R - C <= W).  The T tiles of column tile
// C (its list trimmed to rows <= Cs) load as one batch of up to kSweepBatch
// while the previous column tile's batch is summed.  Grid: one-dimensional
// over (block, observation tile), member tiles of a block adjacent (one XCD).
constexpr int kBwdBatch = 16;

__global__ __launch_bounds__(64) void k_bwd_sweep_ring(const Block *__restrict__ blocks, int og,
                                                       const int64_t *__restrict__ ct_ptr,
                                                       const int32_t *__restrict__ ct_row,
                                                       const int32_t *__restrict__ ct_slot,
                                                       const int32_t *__restrict__ bobs_row,
                                                       const int32_t *__restrict__ ot_jmax,
                                                       const double *__restrict__ tiles,
                                                       const double *__restrict__ tinv, int W,
                                                       double *__restrict__ F) {
  extern __shared__ double ring[];
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / og];
  const int oc = (int)(lg % og);
  if (16 * oc >= B.m) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int o = 16 * oc + c;
  const int jo = o < B.m ? bobs_row[B.obs0 + o] : -1;
  const int ldf = B.ldf;
  double *Fb = F + B.F0;
  const int Cs = ot_jmax[B.ot0 + oc] >> 4;
  for (int C = B.nrt - 1; C > Cs; --C) {
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) Fc[(int64_t)(4 * r + q) * ldf] = 0.0;
  }
  const int64_t *cp = ct_ptr + B.rt0;
  // batch cursor: column tile Cl (descending), its list trimmed to rows <= Cs
  int Cl = Cs;
  auto load_batch = [&](double(&tv)[kBwdBatch][4], int(&rs)[kBwdBatch], int &cnt) {
    const int64_t s0 = cp[Cl];
    int64_t s1 = cp[Cl + 1];
    while (s1 > s0 && ct_row[s1 - 1] > Cs) --s1;
    cnt = (int)(s1 - s0 < kBwdBatch ? s1 - s0 : kBwdBatch);
#pragma unroll
    for (int j = 0; j < kBwdBatch; ++j) {
      if (j < cnt) {
        const double *Tt = tiles + (int64_t)ct_slot[s0 + j] * 256 + q * 16 + c;   // A operand: T_RC(4kc + q, c)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) tv[j][kc] = Tt[64 * kc];
        rs[j] = ct_row[s0 + j];
      }
    }
    --Cl;
    return s1 - s0;
  };
  double ta[kBwdBatch][4], tb[kBwdBatch][4];
  int ra[kBwdBatch], rb[kBwdBatch];
  int na = 0, nb = 0;
  int64_t fulla = load_batch(ta, ra, na), fullb = 0;
  for (int C = Cs; C >= 0; --C) {
    if (C > 0) fullb = load_batch(tb, rb, nb);
    const double *Ti = tinv + (B.rt0 + C) * 256 + q * 16 + c;
    double ti[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ti[kc] = Ti[64 * kc];
    d4 acc0, acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc0[r] = (16 * C + 4 * r + q == jo) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < kBwdBatch; ++j) {
      if (j < na) {
        const double *fr = ring + (ra[j] % W) * 256 + 16 * q + c;   // B operand: F_R(4kc + q, o)
        acc0 = mfma64(-ta[j][0], fr[0], acc0);
        acc1 = mfma64(-ta[j][2], fr[128], acc1);
        acc0 = mfma64(-ta[j][1], fr[64], acc0);
        acc1 = mfma64(-ta[j][3], fr[192], acc1);
      }
    }
    // entries beyond the first batch of a long list: T from memory, F_R from the ring
    for (int64_t t = cp[C] + kBwdBatch; t < cp[C] + fulla; ++t) {
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256 + q * 16 + c;
      const double *fr = ring + (ct_row[t] % W) * 256 + 16 * q + c;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc0 = mfma64(-Tt[64 * kc], fr[64 * kc], acc0);
    }
    const d4 acc = acc0 + acc1;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(ti[kc], acc[kc], out);
    double *slot = ring + (C % W) * 256 + 16 * q + c;
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      slot[64 * r] = out[r];
      Fc[(int64_t)(4 * r + q) * ldf] = out[r];
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < kBwdBatch; ++j) {
      ra[j] = rb[j];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) ta[j][kc] = tb[j][kc];
    }
    na = nb;
    fulla = fullb;
  }
}

// The same backward sweep with the gap ring of k_fwd_sweep_gap: LDS slots
// only for the near run of distances 1..D (slot R mod D) and the block's far
// range lo..hi (slot R mod Wf).  At the end of column tile C the tile that
// enters the far range, F_{C-1+lo} (when it lies in the sweep, at or below
// row tile Cs), goes into its slot: from the near ring when lo = D + 1 (the
// tile F_C replaces), otherwise from memory, where this wavefront wrote it at
// least two column tiles earlier; it is requested one column tile ahead.
// Each column tile loads its own batch of T tiles (one batch of registers,
// against two in k_bwd_sweep_ring), which with the smaller ring lets more
// than one wavefront share a SIMD.
template <int D>
__global__ __launch_bounds__(64) void k_bwd_sweep_gap(const Block *__restrict__ blocks, int og,
                                                      const int64_t *__restrict__ ct_ptr,
                                                      const int32_t *__restrict__ ct_row,
                                                      const int32_t *__restrict__ ct_slot,
                                                      const int32_t *__restrict__ bobs_row,
                                                      const int32_t *__restrict__ ot_jmax,
                                                      const double *__restrict__ tiles,
                                                      const double *__restrict__ tinv, double *__restrict__ F) {
  extern __shared__ double ring[];   // D near slots, then the block's far_w far slots
  double *far = ring + D * 256;
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / og];
  const int oc = (int)(lg % og);
  if (16 * oc >= B.m) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int o = 16 * oc + c;
  const int jo = o < B.m ? bobs_row[B.obs0 + o] : -1;
  const int ldf = B.ldf;
  const int lo = B.far_lo, Wf = B.far_w;
  const bool from_mem = lo > D + 1;
  double *Fb = F + B.F0;
  const int Cs = ot_jmax[B.ot0 + oc] >> 4;
  for (int C = B.nrt - 1; C > Cs; --C) {
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) Fc[(int64_t)(4 * r + q) * ldf] = 0.0;
  }
  // lane (q, c) reads and writes element (4r + q, c) of an F tile
  auto load_f = [&](int R, d4 &v) {
    const double *Fr = Fb + (int64_t)(16 * R) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (R <= Cs) ? Fr[(int64_t)(4 * r + q) * ldf] : 0.0;
  };
  auto zr_of = [&](int R, int C) {
    return (R - C <= D ? ring + (R % D) * 256 : far + (R % Wf) * 256) + 16 * q + c;   // B operand: F_R(4kc + q, o)
  };
  const int64_t *cp = ct_ptr + B.rt0;
  int Cl = Cs;
  auto load_batch = [&](double(&tv)[kBwdBatch][4], int(&rs)[kBwdBatch], int &cnt) {
    const int64_t s0 = cp[Cl];
    int64_t s1 = cp[Cl + 1];
    while (s1 > s0 && ct_row[s1 - 1] > Cs) --s1;
    cnt = (int)(s1 - s0 < kBwdBatch ? s1 - s0 : kBwdBatch);
#pragma unroll
    for (int j = 0; j < kBwdBatch; ++j) {
      if (j < cnt) {
        const double *Tt = tiles + (int64_t)ct_slot[s0 + j] * 256 + q * 16 + c;   // A operand: T_RC(4kc + q, c)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) tv[j][kc] = Tt[64 * kc];
        rs[j] = ct_row[s0 + j];
      }
    }
    --Cl;
    return s1 - s0;
  };
  double ta[kBwdBatch][4];
  int ra[kBwdBatch];
  int na = 0;
  d4 fz = d4{0.0, 0.0, 0.0, 0.0};   // far entry for the end of this column tile: F_{C-1+lo}
  if (Wf > 0 && from_mem) load_f(Cs - 1 + lo, fz);
  for (int C = Cs; C >= 0; --C) {
    const int64_t fulla = load_batch(ta, ra, na);   // this column tile's own batch (one batch of registers)
    d4 fzn = d4{0.0, 0.0, 0.0, 0.0};
    if (Wf > 0 && from_mem && C > 0) load_f(C - 2 + lo, fzn);   // written at column tile C - 2 + lo >= C + 1
    const double *Ti = tinv + (B.rt0 + C) * 256 + q * 16 + c;
    double ti[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ti[kc] = Ti[64 * kc];
    d4 acc0, acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc0[r] = (16 * C + 4 * r + q == jo) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < kBwdBatch; ++j) {
      if (j < na) {
        const double *fr = zr_of(ra[j], C);
        acc0 = mfma64(-ta[j][0], fr[0], acc0);
        acc1 = mfma64(-ta[j][2], fr[128], acc1);
        acc0 = mfma64(-ta[j][1], fr[64], acc0);
        acc1 = mfma64(-ta[j][3], fr[192], acc1);
      }
    }
    // entries beyond the first batch of a long list: T from memory, F_R from the ring
    for (int64_t t = cp[C] + kBwdBatch; t < cp[C] + fulla; ++t) {
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256 + q * 16 + c;
      const double *fr = zr_of(ct_row[t], C);
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc0 = mfma64(-Tt[64 * kc], fr[64 * kc], acc0);
    }
    const d4 acc = acc0 + acc1;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(ti[kc], acc[kc], out);
    wave_lds_sync();   // every read of the slots rewritten below is done
    const int Rf = C - 1 + lo;
    if (Wf > 0 && C > 0 && Rf <= Cs) {
      double *fs = far + (Rf % Wf) * 256 + 16 * q + c;
      if (from_mem) {
#pragma unroll
        for (int r = 0; r < 4; ++r) fs[64 * r] = fz[r];
      } else {   // Rf = C + D: the near slot that F_C takes next
        const double *ns = ring + (Rf % D) * 256 + 16 * q + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) fs[64 * r] = ns[64 * r];
      }
    }
    double *slot = ring + (C % D) * 256 + 16 * q + c;
    double *Fc = Fb + (int64_t)(16 * C) * ldf + 16 * oc + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      slot[64 * r] = out[r];
      Fc[(int64_t)(4 * r + q) * ldf] = out[r];
    }
    wave_lds_sync();
    fz = fzn;
  }
}

// S = R + F^T D F (lower tiles, stride ldf); one wavefront per (block, tile
// column J, chunk of up to 8 tile rows I >= J), on a one-dimensional grid
// numbered so that the wavefronts of a block run on one XCD and share its F
// in L2.  The loads of k-step ks + 1 are issued before the products of ks.
constexpr int kDualSTiles = 8;

__global__ __launch_bounds__(64) void k_dual_S(const Block *__restrict__ blocks, int oc,
                                               const int32_t *__restrict__ bobs_o,
                                               const int32_t *__restrict__ ot_jmax, const double *__restrict__ F,
                                               const double *__restrict__ dvec, const double *__restrict__ r_diag,
                                               double *__restrict__ S) {
  int b, jt;
  block_tile(oc * ((oc + kDualSTiles - 1) / kDualSTiles), b, jt);
  const Block B = blocks[b];
  const int J = jt % oc;
  const int TJ = B.ldf >> 4;
  const int I0 = J + kDualSTiles * (jt / oc);
  if (J >= TJ || I0 >= TJ) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int ldf = B.ldf;
  const double *Fb = F + B.F0;
  d4 acc[kDualSTiles];
#pragma unroll
  for (int I = 0; I < kDualSTiles; ++I) acc[I] = d4{0.0, 0.0, 0.0, 0.0};
  // column tile J of F is zero below its largest observed row
  const int ksteps = (ot_jmax[B.ot0 + J] >> 2) + 1;
  auto load = [&](int ks, double &bv, double(&fv)[kDualSTiles]) {
    const int k = 4 * ks + q;
    const double dk = k < B.n ? dvec[B.row0 + k] : 0.0;
    const double *Fk = Fb + (int64_t)k * ldf + c;
    bv = dk * Fk[16 * J];
#pragma unroll
    for (int i = 0; i < kDualSTiles; ++i) fv[i] = I0 + i < TJ ? Fk[16 * (I0 + i)] : 0.0;
  };
  double bc, fc[kDualSTiles];
  load(0, bc, fc);
  for (int ks = 0; ks < ksteps; ++ks) {
    double bn = 0.0, fn[kDualSTiles];
#pragma unroll
    for (int i = 0; i < kDualSTiles; ++i) fn[i] = 0.0;
    if (ks + 1 < ksteps) load(ks + 1, bn, fn);
#pragma unroll
    for (int i = 0; i < kDualSTiles; ++i)
      if (I0 + i < TJ) acc[i] = mfma64(fc[i], bc, acc[i]);
    bc = bn;
#pragma unroll
    for (int i = 0; i < kDualSTiles; ++i) fc[i] = fn[i];
  }
  double *Sb = S + B.S0;
#pragma unroll
  for (int i = 0; i < kDualSTiles; ++i) {
    const int I = I0 + i;
    if (I < TJ) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * I + 4 * r + q, bb = 16 * J + c;
        double v = acc[i][r];
        if (a == bb) v = a < B.m ? v + r_diag[bobs_o[B.obs0 + a]] : 1.0;
        Sb[(int64_t)a * ldf + bb] = v;
      }
    }
  }
}

// In-place Cholesky of each block's S (m x m lower part, stride ldf), one
// workgroup per block: blocks of more than 128 observations.
__global__ __launch_bounds__(256) void k_dual_chol(const Block *__restrict__ blocks, double *__restrict__ S,
                                                   int32_t *status) {
  __shared__ int bad;
  const Block B = blocks[blockIdx.x];
  const int m = B.m, ld = B.ldf, tid = threadIdx.x;
  double *L = S + B.S0;
  if (tid == 0) bad = 0;
  for (int k = 0; k < m; ++k) {
    __syncthreads();
    if (tid == 0) {
      const double piv = L[(int64_t)k * ld + k];
      if (!(piv > 0.0)) bad = 1;
      else L[(int64_t)k * ld + k] = sqrt(piv);
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) set_error(status, ENKFMC_ENOTSPD, -1 - (int32_t)blockIdx.x);
      return;
    }
    const double lkk = L[(int64_t)k * ld + k];
    for (int i = k + 1 + tid; i < m; i += 256) L[(int64_t)i * ld + k] /= lkk;
    __syncthreads();
    const int t = m - k - 1;
    for (int64_t idx = tid; idx < (int64_t)t * t; idx += 256) {
      const int i = k + 1 + (int)(idx / t), j = k + 1 + (int)(idx % t);
      if (j <= i) L[(int64_t)i * ld + j] -= L[(int64_t)i * ld + k] * L[(int64_t)j * ld + k];
    }
  }
}

// Q = S^-1 Delta, one lane per member column; rows m..ldf-1 of Q are zeroed.
template <typename TX>
__global__ __launch_bounds__(64) void k_dual_Q(const Block *__restrict__ blocks, const int32_t *__restrict__ bobs_o,
                                               const int32_t *__restrict__ bobs_row,
                                               const int32_t *__restrict__ fit_glob, const double *__restrict__ S,
                                               const double *__restrict__ Y, const TX *__restrict__ Xb, int64_t ld,
                                               int N, double *__restrict__ Q) {
  const Block B = blocks[blockIdx.x];
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= N || B.m == 0) return;
  const int m = B.m, lds = B.ldf;
  const double *L = S + B.S0;
  double *q = Q + B.Q0;
  for (int a = 0; a < m; ++a) {
    const int o = bobs_o[B.obs0 + a];
    const int64_t g = fit_glob[B.row0 + bobs_row[B.obs0 + a]];
    q[(int64_t)a * N + c] = Y[(int64_t)o * N + c] - (double)Xb[g * ld + c];
  }
  chol_solve_col(L, lds, m, q + c, N);
  for (int a = m; a < lds; ++a) q[(int64_t)a * N + c] = 0.0;
}

// X = S^-1 V for one block and one tile of 16 members, from the Cholesky
// factor L of S that k_dual_chol* leave in S (lower triangle, row stride
// ldf): forward L Y = V, then backward L^T X = Y, by 16-row tiles.  The
// products with the other tiles run on the matrix cores, their L operands
// loaded straight from S (held in L2 for the block's member tiles, which are
// neighbouring workgroups).  Inside a diagonal tile the 16 rows are taken in
// turn from an LDS copy of the tile whose diagonal and upper part are zeroed,
// 1/L_kk kept beside it.  Rows are permuted inside every tile: row 4q + r of
// a tile sits at lane (q, c), register r (member c), and MFMA row rho = 4r + q
// stands for it on both sides of every product, so a lane's A operands of
// L_IJ are four consecutive doubles of one row.  Rows at or past m are zero
// throughout (their loads masked), and rows m..ldf-1 of the result are
// written as zeros.
// MODE 0: V = Y^s - H X_b, X to Q (the analysis); MODE 1: V = Q, solved in
// place (the reverse pass).
constexpr int kSolveMaxTiles = 8;   // blocks of up to 128 observations

// quarter_bcast with the row as an argument (a constant once the loops that
// call it are unrolled)
__device__ __forceinline__ double quarter_bcast_n(double v, int Q) {
  switch (Q) {
    case 0: return quarter_bcast<0>(v);
    case 1: return quarter_bcast<1>(v);
    case 2: return quarter_bcast<2>(v);
    default: return quarter_bcast<3>(v);
  }
}

template <int MODE, typename TX>
__global__ __launch_bounds__(64) void k_solve_S_tiles(const Block *__restrict__ blocks, int G,
                                                      const int32_t *__restrict__ bobs_o,
                                                      const int32_t *__restrict__ bobs_row,
                                                      const int32_t *__restrict__ fit_glob,
                                                      const double *__restrict__ S, const double *__restrict__ Y,
                                                      const TX *__restrict__ Xb, int64_t ld, int N,
                                                      double *__restrict__ Q) {
  __shared__ double dt[256];
  __shared__ double dinv[16];
  int b, g;
  block_tile(G, b, g);
  const Block B = blocks[b];
  const int m = B.m;
  if (m == 0) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int pc = 4 * (c & 3) + (c >> 2);   // the tile row that MFMA row c stands for
  const int col = 16 * g + c;
  const bool cok = col < N;
  const int TT = (m + 15) >> 4, ldf = B.ldf;
  const double *L = S + B.S0;
  double *Qb = Q + B.Q0;
  d4 y[kSolveMaxTiles];
#pragma unroll
  for (int I = 0; I < kSolveMaxTiles; ++I) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = 16 * I + 4 * q + r;
      double v = 0.0;
      if (I < TT && a < m && cok) {
        if constexpr (MODE == 0) {
          const int o = bobs_o[B.obs0 + a];
          const int64_t gl = fit_glob[B.row0 + bobs_row[B.obs0 + a]];
          v = Y[(int64_t)o * N + col] - (double)Xb[gl * ld + col];
        } else {
          v = Qb[(int64_t)a * N + col];
        }
      }
      y[I][r] = v;
    }
  }
  // diagonal tile I to LDS: lane l takes row l >> 2, columns 4 (l & 3) .. + 3
  auto stage = [&](int I) {
    const int rr = lane >> 2, c0 = 4 * (lane & 3), ar = 16 * I + rr;
    const double *src = L + (int64_t)ar * ldf + 16 * I + c0;
    const double2 v01 = *(const double2 *)src, v23 = *(const double2 *)(src + 2);
    const double vv[4] = {v01.x, v01.y, v23.x, v23.y};
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = c0 + j;
      dt[rr * 16 + cc] = (cc < rr && ar < m) ? vv[j] : 0.0;
      if (cc == rr) dinv[rr] = ar < m ? 1.0 / vv[j] : 1.0;
    }
    wave_lds_sync();
  };
  // forward: Y_I = L_II^-1 (V_I - sum_{J<I} L_IJ Y_J)
#pragma unroll
  for (int I = 0; I < kSolveMaxTiles; ++I) {
    if (I < TT) {
      d4 t = y[I];
      const int arow = 16 * I + pc;
      const bool rok = arow < m;
#pragma unroll
      for (int J = 0; J < I; ++J) {
        const double *src = L + (int64_t)arow * ldf + 16 * J + 4 * q;
        const double2 a01 = *(const double2 *)src, a23 = *(const double2 *)(src + 2);
        t = mfma64(rok ? -a01.x : 0.0, y[J][0], t);
        t = mfma64(rok ? -a01.y : 0.0, y[J][1], t);
        t = mfma64(rok ? -a23.x : 0.0, y[J][2], t);
        t = mfma64(rok ? -a23.y : 0.0, y[J][3], t);
      }
      stage(I);
#pragma unroll
      for (int k = 0; k < 16; ++k) {   // row k is final here: it sits at lanes q = k / 4, register k % 4
        const double yk = quarter_bcast_n(t[k & 3] * dinv[k], k >> 2);
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = fma(-dt[(4 * q + r) * 16 + k], yk, t[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) y[I][r] = t[r] * dinv[4 * q + r];
    }
  }
  // backward: X_I = L_II^-T (Y_I - sum_{J>I} L_JI^T X_J)
#pragma unroll
  for (int I = kSolveMaxTiles - 1; I >= 0; --I) {
    if (I < TT) {
      d4 t = y[I];
#pragma unroll
      for (int J = I + 1; J < kSolveMaxTiles; ++J) {
        if (J < TT) {
          const double *src = L + (int64_t)(16 * J + 4 * q) * ldf + 16 * I + pc;
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const double v = src[(int64_t)kc * ldf];
            t = mfma64(16 * J + 4 * q + kc < m ? -v : 0.0, y[J][kc], t);
          }
        }
      }
      stage(I);
#pragma unroll
      for (int k = 15; k >= 0; --k) {
        const double xk = quarter_bcast_n(t[k & 3] * dinv[k], k >> 2);
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = fma(-dt[k * 16 + 4 * q + r], xk, t[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) y[I][r] = t[r] * dinv[4 * q + r];
    }
  }
  if (cok) {
#pragma unroll
    for (int I = 0; I < kSolveMaxTiles; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * I + 4 * q + r;
        if (a < ldf) Qb[(int64_t)a * N + col] = I < TT ? y[I][r] : 0.0;
      }
  }
}

template <typename TX>
static void launch_solve_S(enkfmc_plan *p, const Dev &d, int mode, const TX *Xb, int64_t ld, const double *Y,
                           double *Q, hipStream_t s) {
  const int G = (p->N + 15) / 16;
  const dim3 grid((unsigned)(p->blocks.size() * G));
  if (mode == 0)
    hipLaunchKernelGGL((k_solve_S_tiles<0, TX>), grid, dim3(64), 0, s, d.blocks, G, d.bobs_o, d.bobs_row, d.fit_glob,
                       d.S, Y, Xb, ld, p->N, Q);
  else
    hipLaunchKernelGGL((k_solve_S_tiles<1, TX>), grid, dim3(64), 0, s, d.blocks, G, d.bobs_o, d.bobs_row, d.fit_glob,
                       d.S, Y, Xb, ld, p->N, Q);
}

bool solve_S_tiles_fit(const enkfmc_plan *p) { return p->max_bm <= 16 * kSolveMaxTiles; }

hipError_t launch_adj_solve_S_tiles(enkfmc_plan *p, const Dev &d, double *P, hipStream_t s) {
  launch_solve_S<double>(p, d, 1, nullptr, 0, nullptr, P, s);
  return hipGetLastError();
}

// G = D (F Q) of row tile R (or D (V - F Q) with V given), written into the
// output rows that the forward sweep then solves in place.  One wavefront per
// (block, row tile).  Each F fragment it loads feeds up to kGTiles 16-member
// column tiles at once, so F_R is read once per kGTiles member tiles.  (A
// one-dimensional grid with the row tiles of a block on one XCD, as in
// k_dual_S, was slower here: 1.37 ms against 1.30 at T-63.)
constexpr int kGTiles = 5;

__global__ __launch_bounds__(64) void k_dual_G(const Block *__restrict__ blocks, const int32_t *__restrict__ ot_jmax,
                                               const double *__restrict__ F, const double *__restrict__ Q,
                                               const double *__restrict__ dvec, const double *__restrict__ V, int N,
                                               double *__restrict__ G) {
  const Block B = blocks[blockIdx.x];
  const int R = blockIdx.y;
  if (R >= B.nrt) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int ldf = B.ldf;
  const double *Fr = F + B.F0 + (int64_t)(16 * R + c) * ldf + q;
  const double *Qb = Q + B.Q0;
  double dd[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * R + 4 * r + q;
    dd[r] = row < B.n ? dvec[B.row0 + row] : 0.0;
  }
  const int ng = (N + 15) >> 4;
  for (int g0 = 0; g0 < ng; g0 += kGTiles) {
    const int ngc = ng - g0 < kGTiles ? ng - g0 : kGTiles;
    d4 acc[kGTiles];
#pragma unroll
    for (int g = 0; g < kGTiles; ++g) acc[g] = d4{0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < (ldf >> 4); ++t) {
      if (ot_jmax[B.ot0 + t] < 16 * R) continue;   // F_R is zero in these 16 columns
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int ks = 4 * t + kk;
        const double fa = Fr[4 * ks];
        const double *qr = Qb + (int64_t)(4 * ks + q) * N;
#pragma unroll
        for (int g = 0; g < kGTiles; ++g) {
          if (g < ngc) {
            const int colj = 16 * (g0 + g) + c;
            const double bq = qr[colj < N ? colj : 0];   // clamped: the address stays inside the row
            acc[g] = mfma64(fa, colj < N ? bq : 0.0, acc[g]);
          }
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kGTiles; ++g) {
      const int colj = 16 * (g0 + g) + c;
      if (g >= ngc || colj >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * R + 4 * r + q;
        if (row < B.n) {
          const int64_t o = (B.row0 + row) * N + colj;
          G[o] = V ? dd[r] * (V[o] - acc[g][r]) : dd[r] * acc[g][r];
        }
      }
    }
  }
}

// Z = T^-1 G in place (G from k_dual_G), forward over row tiles; one wavefront
// per (block, 16 member columns).  Row tile R: Z_R = T_RR^-1 (G_R - sum_C T_RC Z_C).
__global__ __launch_bounds__(64) void k_fwd_sweep(const Block *__restrict__ blocks, const int64_t *__restrict__ rt_ptr,
                                                  const int32_t *__restrict__ rt_col,
                                                  const int32_t *__restrict__ rt_slot,
                                                  const double *__restrict__ tiles, const double *__restrict__ tinv,
                                                  int N, double *__restrict__ Z) {
  const Block B = blocks[blockIdx.x];
  const int cc = blockIdx.y;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  const int coll = colok ? colj : 0;
  double *Zb = Z + B.row0 * N;
  for (int R = 0; R < B.nrt; ++R) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * R + 4 * r + q;
      acc[r] = (row < B.n && colok) ? Zb[(int64_t)row * N + colj] : 0.0;
    }
    const int64_t s0 = rt_ptr[B.rt0 + R], s1 = rt_ptr[B.rt0 + R + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int C = rt_col[t];
      const double *Tt = tiles + (int64_t)rt_slot[t] * 256 + c * 16 + q;
      const double *Zc = Zb + (int64_t)(16 * C + q) * N + coll;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double z = Zc[(int64_t)(4 * kc) * N];
        acc = mfma64(-Tt[4 * kc], colok ? z : 0.0, acc);
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
        if (row < B.n) Zb[(int64_t)row * N + colj] = out[r];
      }
    }
  }
}

// The same sweep with this wavefront's last W row tiles of Z kept in LDS, a
// ring of 16x16 tiles (row-major) where row tile R sits at slot R mod W.  Every
// stored T_RC has R - C <= W (W is the plan's largest such distance), so each
// product T_RC Z_C reads Z_C from the ring rather than from memory.  The T
// tiles of a row tile are taken in batches of up to kSweepBatch, and the next
// batch (of this row tile or the next) loads while the current one is summed;
// G and the inverse diagonal tile of the next row tile load one row tile
// ahead.  The four k-steps of a tile go to two accumulators, halving the
// dependent MFMA chain.  The grid is one-dimensional over (block, member
// tile), numbered so that the member tiles of a block run on one XCD and share
// its T tiles in L2.
constexpr int kSweepBatch = 16;

__global__ __launch_bounds__(64) void k_fwd_sweep_ring(const Block *__restrict__ blocks, int ng,
                                                       const int64_t *__restrict__ rt_ptr,
                                                       const int32_t *__restrict__ rt_col,
                                                       const int32_t *__restrict__ rt_slot,
                                                       const double *__restrict__ tiles,
                                                       const double *__restrict__ tinv, int N, int W,
                                                       double *__restrict__ Z) {
  extern __shared__ double ring[];
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / ng];
  const int cc = (int)(lg % ng);
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  double *Zb = Z + B.row0 * N;
  if (B.nrt <= 0) return;
  const int64_t *rp = rt_ptr + B.rt0;
  auto load_g = [&](int R, d4 &g, double(&ti)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * R + 4 * r + q;
      g[r] = (row < B.n && colok) ? Zb[(int64_t)row * N + colj] : 0.0;
    }
    const double *Ti = tinv + (B.rt0 + R) * 256 + c * 16 + q;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ti[kc] = Ti[4 * kc];
  };
  // batch cursor: row tile Rl, next tile tl of its list
  int Rl = 0;
  int64_t tl = rp[0];
  auto load_batch = [&](double(&tv)[kSweepBatch][4], int(&cs)[kSweepBatch], int &cnt, int &R, bool &last) {
    const int64_t end = rp[Rl + 1];
    cnt = (int)(end - tl < kSweepBatch ? end - tl : kSweepBatch);
    R = Rl;
#pragma unroll
    for (int j = 0; j < kSweepBatch; ++j) {
      if (j < cnt) {
        const double *Tt = tiles + (int64_t)rt_slot[tl + j] * 256 + c * 16 + q;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) tv[j][kc] = Tt[4 * kc];
        cs[j] = rt_col[tl + j];
      }
    }
    tl += cnt;
    last = tl == end;
    if (last) ++Rl;
  };
  double ta[kSweepBatch][4], tb[kSweepBatch][4];
  int ca[kSweepBatch], cb[kSweepBatch];
  int na = 0, nb = 0, Ra = 0, Rb = 0;
  bool la = true, lb = true;
  load_batch(ta, ca, na, Ra, la);
  d4 acc0, acc1 = d4{0.0, 0.0, 0.0, 0.0}, gn = d4{0.0, 0.0, 0.0, 0.0};
  double ti[4], tin[4] = {0.0, 0.0, 0.0, 0.0};
  load_g(0, acc0, ti);
  if (B.nrt > 1) load_g(1, gn, tin);
  while (true) {
    const bool more = Rl < B.nrt;
    if (more) load_batch(tb, cb, nb, Rb, lb);
#pragma unroll
    for (int j = 0; j < kSweepBatch; ++j) {
      if (j < na) {
        const double *zr = ring + (ca[j] % W) * 256 + 16 * q + c;   // B operand: Z_C(4kc + q, c)
        acc0 = mfma64(-ta[j][0], zr[0], acc0);
        acc1 = mfma64(-ta[j][2], zr[128], acc1);
        acc0 = mfma64(-ta[j][1], zr[64], acc0);
        acc1 = mfma64(-ta[j][3], zr[192], acc1);
      }
    }
    if (la) {
      // row tile Ra is complete: Z_Ra = T_RaRa^-1 (G_Ra - sum_C T_RaC Z_C)
      const d4 acc = acc0 + acc1;
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) out = mfma64(ti[kc], acc[kc], out);
      double *slot = ring + (Ra % W) * 256 + 16 * q + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        slot[64 * r] = out[r];
        const int row = 16 * Ra + 4 * r + q;
        if (colok && row < B.n) Zb[(int64_t)row * N + colj] = out[r];
      }
      wave_lds_sync();
      if (Ra + 1 >= B.nrt) break;
      acc0 = gn;
      acc1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) ti[kc] = tin[kc];
      if (Ra + 2 < B.nrt) load_g(Ra + 2, gn, tin);
    }
    // every row tile ends a batch, so a batch remains while row tiles do
#pragma unroll
    for (int j = 0; j < kSweepBatch; ++j) {
      ca[j] = cb[j];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) ta[j][kc] = tb[j][kc];
    }
    na = nb;
    Ra = Rb;
    la = lb;
  }
}

// The forward sweep split by tile distance.  With D the plan's near distance
// (every distance 1..D occurs, the stored tiles further back are "far"),
// the row tiles go in chunks of D + 1: a far tile T_RC of a chunk's row tile
// has C in an earlier chunk, so the far sums G_R - sum_far T_RC Z_C of the
// whole chunk are independent products, read from memory, accumulated in
// registers at the chunk's start; the near tiles follow row tile by row tile
// from a ring of the last D Z tiles in LDS (D x 2 KB, not the largest
// distance x 2 KB of k_fwd_sweep_ring), so several chains share a SIMD.  The
// far T rows are loaded four consecutive doubles per lane (k-step kc takes
// column 4q + kc).  One wavefront per (block, member tile).
template <int D>
__global__ __launch_bounds__(64) void k_fwd_sweep_near(const Block *__restrict__ blocks, int ng,
                                                       const int64_t *__restrict__ rt_ptr,
                                                       const int32_t *__restrict__ rt_col,
                                                       const int32_t *__restrict__ rt_slot,
                                                       const int32_t *__restrict__ rt_nfar,
                                                       const double *__restrict__ tiles,
                                                       const double *__restrict__ tinv, int N,
                                                       double *__restrict__ Z) {
  constexpr int W = D + 1;
  constexpr int kFarBatch = 4;   // far tiles whose loads are issued together
  __shared__ double ring[D * 256];
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / ng];
  const int cc = (int)(lg % ng);
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  double *Zb = Z + B.row0 * N;
  const int64_t *rp = rt_ptr + B.rt0;
  for (int k0 = 0; k0 < B.nrt; k0 += W) {
    d4 acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int R = k0 + j;
      acc[j] = d4{0.0, 0.0, 0.0, 0.0};
      if (R >= B.nrt) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * R + 4 * r + q;
        acc[j][r] = (row < B.n && colok) ? Zb[(int64_t)row * N + colj] : 0.0;   // G_R
      }
      // far tiles (the first rt_nfar of the ascending list, C < R - D): Z_C
      // from memory, kFarBatch tiles' loads issued before their products
      const int64_t tf0 = rp[R], tf1 = tf0 + rt_nfar[B.rt0 + R];
      for (int64_t tb = tf0; tb < tf1; tb += kFarBatch) {
        double ta[kFarBatch][4], zv[kFarBatch][4];
#pragma unroll
        for (int u = 0; u < kFarBatch; ++u) {
          const bool in = tb + u < tf1;
          const int64_t t = in ? tb + u : tf0;
          const int C = rt_col[t];
          const d2 *Tt = (const d2 *)(tiles + (int64_t)rt_slot[t] * 256 + c * 16 + 4 * q);   // A: T_RC(c, 4q + kc)
          const d2 lo = Tt[0], hi = Tt[1];
          ta[u][0] = in ? lo[0] : 0.0; ta[u][1] = in ? lo[1] : 0.0;
          ta[u][2] = in ? hi[0] : 0.0; ta[u][3] = in ? hi[1] : 0.0;
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const int row = 16 * C + 4 * q + kc;   // B: Z_C(4q + kc, c)
            zv[u][kc] = (row < B.n && colok) ? Zb[(int64_t)row * N + colj] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < kFarBatch; ++u)
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) acc[j] = mfma64(-ta[u][kc], zv[u][kc], acc[j]);
      }
    }
    // near tiles, row tile by row tile
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int R = k0 + j;
      if (R >= B.nrt) break;
      d4 a0 = acc[j], a1 = d4{0.0, 0.0, 0.0, 0.0};
      // near tiles (at most D, distances 1..D): their loads issued together
      const int64_t tn0 = rp[R] + rt_nfar[B.rt0 + R], tn1 = rp[R + 1];
      d2 nlo[D], nhi[D];
      int ncol[D];
#pragma unroll
      for (int u = 0; u < D; ++u) {
        ncol[u] = -1;
        nlo[u] = nhi[u] = d2{0.0, 0.0};
        if (tn0 + u < tn1) {   // uniform over the wavefront
          ncol[u] = rt_col[tn0 + u];
          const d2 *Tt = (const d2 *)(tiles + (int64_t)rt_slot[tn0 + u] * 256 + c * 16 + 4 * q);
          nlo[u] = Tt[0];
          nhi[u] = Tt[1];
        }
      }
#pragma unroll
      for (int u = 0; u < D; ++u) {
        if (ncol[u] < 0) break;
        const double *zr = ring + (ncol[u] % D) * 256 + 64 * q + c;   // B operand: Z_C(4q + kc, c)
        a0 = mfma64(-nlo[u][0], zr[0], a0);
        a1 = mfma64(-nhi[u][0], zr[32], a1);
        a0 = mfma64(-nlo[u][1], zr[16], a0);
        a1 = mfma64(-nhi[u][1], zr[48], a1);
      }
      const d4 sum = a0 + a1;
      // Z_R = T_RR^-1 (G_R - sum_C T_RC Z_C)
      const double *Ti = tinv + (B.rt0 + R) * 256 + c * 16 + q;
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) out = mfma64(Ti[4 * kc], sum[kc], out);
      wave_lds_sync();   // every read of the slot's previous tile (Z_{R-D}) is done
      double *slot = ring + (R % D) * 256 + 16 * q + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        slot[64 * r] = out[r];
        const int row = 16 * R + 4 * r + q;
        if (colok && row < B.n) Zb[(int64_t)row * N + colj] = out[r];
      }
      wave_lds_sync();
    }
  }
}

// The forward sweep with a ring of only the Z tiles that stored tiles reach:
// the near run of distances 1..D (slot C mod D) and the block's far range
// lo..hi (slot C mod Wf, Wf = hi - lo + 1, from the planner), leaving out the
// distances between them, which none of the block's tiles has.  Each product reads its Z tile from LDS.  At the
// end of row tile R the tile entering the far range, Z_{R+1-lo}, goes into
// its slot: from the near ring when lo = D + 1 (it is the tile Z_R is about
// to replace), otherwise from memory, where this wavefront wrote it at least
// two row tiles earlier.  So each Z tile comes back from memory at most once,
// where the split sweep reads it once per far tile that uses it.  A row
// tile's T tiles load together, kGapBatch at a time; G, the inverse diagonal
// tile and the far entry of the next row tile load one row tile ahead.  One
// wavefront per (block, member tile), numbered so that the member tiles of a
// block share its T tiles in L2.
constexpr int kGapBatch = 16;

template <int D>
__global__ __launch_bounds__(64) void k_fwd_sweep_gap(const Block *__restrict__ blocks, int ng,
                                                      const int64_t *__restrict__ rt_ptr,
                                                      const int32_t *__restrict__ rt_col,
                                                      const int32_t *__restrict__ rt_slot,
                                                      const double *__restrict__ tiles,
                                                      const double *__restrict__ tinv, int N,
                                                      double *__restrict__ Z) {
  extern __shared__ double ring[];   // D near slots, then the block's far_w far slots
  double *far = ring + D * 256;
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / ng];
  const int cc = (int)(lg % ng);
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  double *Zb = Z + B.row0 * N;
  const int64_t *rp = rt_ptr + B.rt0;
  const int lo = B.far_lo, Wf = B.far_w;
  const bool from_mem = lo > D + 1;
  // lane (q, c) reads and writes element (4r + q, c) of a Z tile (row 16R + 4r + q)
  auto load_z = [&](int R, d4 &v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * R + 4 * r + q;
      v[r] = (R >= 0 && row < B.n && colok) ? Zb[(int64_t)row * N + colj] : 0.0;
    }
  };
  auto load_ti = [&](int R, double(&ti)[4]) {
    const double *Ti = tinv + (B.rt0 + R) * 256 + c * 16 + q;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ti[kc] = Ti[4 * kc];
  };
  d4 g, fz = d4{0.0, 0.0, 0.0, 0.0};
  double ti[4];
  load_z(0, g);
  load_ti(0, ti);
  if (Wf > 0 && from_mem) load_z(1 - lo, fz);
  for (int R = 0; R < B.nrt; ++R) {
    // the next row tile's G, inverse diagonal tile and far entry, one row tile ahead
    d4 gn = d4{0.0, 0.0, 0.0, 0.0}, fzn = d4{0.0, 0.0, 0.0, 0.0};
    double tin[4] = {0.0, 0.0, 0.0, 0.0};
    if (R + 1 < B.nrt) {
      load_z(R + 1, gn);
      load_ti(R + 1, tin);
      if (Wf > 0 && from_mem) load_z(R + 2 - lo, fzn);   // written at row tile R + 2 - lo <= R - 1
    }
    d4 a0 = g, a1 = d4{0.0, 0.0, 0.0, 0.0};
    const int64_t t1 = rp[R + 1];
    for (int64_t tb = rp[R]; tb < t1; tb += kGapBatch) {
      d2 tl[kGapBatch], th[kGapBatch];
      int cs[kGapBatch];
#pragma unroll
      for (int u = 0; u < kGapBatch; ++u) {
        cs[u] = -1;
        if (tb + u < t1) {   // uniform over the wavefront
          cs[u] = rt_col[tb + u];
          const d2 *Tt = (const d2 *)(tiles + (int64_t)rt_slot[tb + u] * 256 + c * 16 + 4 * q);   // A: T_RC(c, 4q + kc)
          tl[u] = Tt[0];
          th[u] = Tt[1];
        }
      }
#pragma unroll
      for (int u = 0; u < kGapBatch; ++u) {
        if (cs[u] < 0) break;
        const int C = cs[u];
        const double *zr = (R - C <= D ? ring + (C % D) * 256 : far + (C % Wf) * 256) + 64 * q + c;   // B: Z_C(4q + kc, c)
        a0 = mfma64(-tl[u][0], zr[0], a0);
        a1 = mfma64(-th[u][0], zr[32], a1);
        a0 = mfma64(-tl[u][1], zr[16], a0);
        a1 = mfma64(-th[u][1], zr[48], a1);
      }
    }
    // Z_R = T_RR^-1 (G_R - sum_C T_RC Z_C)
    const d4 sum = a0 + a1;
    d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) out = mfma64(ti[kc], sum[kc], out);
    wave_lds_sync();   // every read of the slots rewritten below is done
    const int Cf = R + 1 - lo;
    if (Wf > 0 && Cf >= 0) {
      double *fs = far + (Cf % Wf) * 256 + 16 * q + c;
      if (from_mem) {
#pragma unroll
        for (int r = 0; r < 4; ++r) fs[64 * r] = fz[r];
      } else {   // Cf = R - D: the near slot that Z_R takes next
        const double *ns = ring + (Cf % D) * 256 + 16 * q + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) fs[64 * r] = ns[64 * r];
      }
    }
    double *slot = ring + (R % D) * 256 + 16 * q + c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      slot[64 * r] = out[r];
      const int row = 16 * R + 4 * r + q;
      if (colok && row < B.n) Zb[(int64_t)row * N + colj] = out[r];
    }
    wave_lds_sync();
    g = gn;
    fz = fzn;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ti[kc] = tin[kc];
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

int max_block_tiles(const enkfmc_plan *p) {
  int mx = 0;
  for (const Block &B : p->blocks) mx = B.nrt > mx ? B.nrt : mx;
  return mx;
}

// Inverse of every diagonal tile, (I + L)^-1 with L its strictly lower part
// (tdiag), when the fit has written the tiles itself: 16 row tiles per
// workgroup, staged in LDS, 16 lanes each (column j by forward substitution,
// the same arithmetic as k_build_tiles).
__global__ __launch_bounds__(256) void k_tile_inverse(const double *__restrict__ tdiag, int64_t n_rt,
                                                      double *__restrict__ tinv) {
  __shared__ double sd[16 * 256];
  const int grp = threadIdx.x >> 4, j = threadIdx.x & 15;
  const int64_t base = (int64_t)blockIdx.x * 16;
  for (int e = threadIdx.x; e < 16 * 256; e += 256) {
    const int64_t t = base + (e >> 8);
    sd[e] = t < n_rt ? tdiag[t * 256 + (e & 255)] : 0.0;
  }
  __syncthreads();
  const int64_t rt = base + grp;
  if (rt >= n_rt) return;
  const double *diag = sd + grp * 256;
  double x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) v -= diag[i * 16 + k] * x[k];
    x[i] = (i < j) ? 0.0 : v;
  }
  double *dst = tinv + rt * 256;
#pragma unroll
  for (int i = 0; i < 16; ++i) dst[i * 16 + j] = x[i];
}

hipError_t launch_tile_inverse(enkfmc_plan *p, const Dev &d, hipStream_t s) {
  phase_begin(p, ENKFMC_PH_TILES, s);
  if (p->n_rt > 0)
    hipLaunchKernelGGL(k_tile_inverse, dim3((unsigned)((p->n_rt + 15) / 16)), dim3(256), 0, s, d.tdiag,
                       (int64_t)p->n_rt, d.tinv);
  phase_end(p, ENKFMC_PH_TILES, s);
  return hipGetLastError();
}

hipError_t launch_build_tiles(enkfmc_plan *p, const Dev &d, hipStream_t s) {
  phase_begin(p, ENKFMC_PH_TILES, s);
  hipLaunchKernelGGL(k_build_tiles, dim3((unsigned)p->blocks.size(), (unsigned)max_block_tiles(p)), dim3(64), 0, s,
                     d.blocks, d.row_ptr, d.col, d.tval, d.rt_ptr, d.rt_col, d.rt_slot, d.tiles, d.tinv, d.tdiag);
  phase_end(p, ENKFMC_PH_TILES, s);
  return hipGetLastError();
}

hipError_t launch_fwd_sweep(enkfmc_plan *p, const Dev &d, const double *Q, const double *V, double *out,
                            hipStream_t s) {
  const unsigned nb = (unsigned)p->blocks.size();
  phase_begin(p, ENKFMC_PH_DUAL_G, s);
  hipLaunchKernelGGL(k_dual_G, dim3(nb, (unsigned)max_block_tiles(p)), dim3(64), 0, s, d.blocks, d.ot_jmax, d.F, Q,
                     d.dvec, V, p->N, out);
  phase_end(p, ENKFMC_PH_DUAL_G, s);
  phase_begin(p, ENKFMC_PH_SWEEP, s);
  const int ng = (p->N + 15) / 16;
  const int W = std::max(1, (int)p->max_rt_back);
#define FWD_NEAR(DD)                                                                                           \
  hipLaunchKernelGGL(k_fwd_sweep_near<DD>, dim3(nb * (unsigned)ng), dim3(64), 0, s, d.blocks, ng, d.rt_ptr,     \
                     d.rt_col, d.rt_slot, d.rt_nfar, d.tiles, d.tinv, p->N, out)
  const size_t gap_bytes = (size_t)(p->near_d + p->far_w) * 2048;
#define FWD_GAP(DD)                                                                                            \
  hipLaunchKernelGGL(k_fwd_sweep_gap<DD>, dim3(nb * (unsigned)ng), dim3(64), gap_bytes, s, d.blocks, ng,       \
                     d.rt_ptr, d.rt_col, d.rt_slot, d.tiles, d.tinv, p->N, out)
  if (p->near_d < W && gap_bytes <= kGapRingMaxBytes) {   // far tiles within a small ring: the gap sweep
    switch (p->near_d) {
      case 1: FWD_GAP(1); break;
      case 2: FWD_GAP(2); break;
      case 3: FWD_GAP(3); break;
      case 4: FWD_GAP(4); break;
      case 5: FWD_GAP(5); break;
      case 6: FWD_GAP(6); break;
      case 7: FWD_GAP(7); break;
      default: FWD_GAP(8); break;
    }
  } else if (p->near_d < W) {   // far tiles exist: the split sweep
    switch (p->near_d) {
      case 1: FWD_NEAR(1); break;
      case 2: FWD_NEAR(2); break;
      case 3: FWD_NEAR(3); break;
      case 4: FWD_NEAR(4); break;
      case 5: FWD_NEAR(5); break;
      case 6: FWD_NEAR(6); break;
      case 7: FWD_NEAR(7); break;
      default: FWD_NEAR(8); break;
    }
  } else if ((size_t)W * 2048 <= kRingMaxBytes)
    hipLaunchKernelGGL(k_fwd_sweep_ring, dim3(nb * (unsigned)ng), dim3(64), (size_t)W * 2048, s, d.blocks, ng,
                       d.rt_ptr, d.rt_col, d.rt_slot, d.tiles, d.tinv, p->N, W, out);
  else
    hipLaunchKernelGGL(k_fwd_sweep, dim3(nb, (unsigned)ng), dim3(64), 0, s, d.blocks, d.rt_ptr, d.rt_col, d.rt_slot,
                       d.tiles, d.tinv, p->N, out);
#undef FWD_NEAR
#undef FWD_GAP
  phase_end(p, ENKFMC_PH_SWEEP, s);
  return hipGetLastError();
}

// F = T^-T H^T, S = R + F^T D F and the Cholesky factor of S of every block
// (the parts of the dual form that do not depend on the innovations).
hipError_t launch_dual_factor(enkfmc_plan *p, const Dev &d, const double *r_diag, hipStream_t s) {
  const unsigned nb = (unsigned)p->blocks.size();
  const unsigned oc = (unsigned)((p->max_bm + 15) / 16);
  if (p->max_bm > 0) {
    phase_begin(p, ENKFMC_PH_DUAL_F, s);
    const int W = std::max(1, (int)p->max_rt_back);
    const size_t gap_bytes = (size_t)(p->near_d + p->far_w) * 2048;
#define BWD_GAP(DD)                                                                                            \
  hipLaunchKernelGGL(k_bwd_sweep_gap<DD>, dim3(nb * oc), dim3(64), gap_bytes, s, d.blocks, (int)oc, d.ct_ptr,  \
                     d.ct_row, d.ct_slot, d.bobs_row, d.ot_jmax, d.tiles, d.tinv, d.F)
    if (p->near_d < W && gap_bytes <= kGapRingMaxBytes) {
      switch (p->near_d) {
        case 1: BWD_GAP(1); break;
        case 2: BWD_GAP(2); break;
        case 3: BWD_GAP(3); break;
        case 4: BWD_GAP(4); break;
        case 5: BWD_GAP(5); break;
        case 6: BWD_GAP(6); break;
        case 7: BWD_GAP(7); break;
        default: BWD_GAP(8); break;
      }
    } else if ((size_t)W * 2048 <= kRingMaxBytes)
      hipLaunchKernelGGL(k_bwd_sweep_ring, dim3(nb * oc), dim3(64), (size_t)W * 2048, s, d.blocks, (int)oc, d.ct_ptr,
                         d.ct_row, d.ct_slot, d.bobs_row, d.ot_jmax, d.tiles, d.tinv, W, d.F);
    else
      hipLaunchKernelGGL(k_bwd_sweep, dim3(nb, oc), dim3(64), 0, s, d.blocks, d.ct_ptr, d.ct_row, d.ct_slot,
                         d.bobs_row, d.ot_jmax, d.tiles, d.tinv, d.F);
#undef BWD_GAP
    phase_end(p, ENKFMC_PH_DUAL_F, s);
    phase_begin(p, ENKFMC_PH_DUAL_S, s);
    hipLaunchKernelGGL(k_dual_S, dim3(nb * oc * ((oc + kDualSTiles - 1) / kDualSTiles)), dim3(64), 0, s, d.blocks,
                       (int)oc, d.bobs_o, d.ot_jmax, d.F, d.dvec, r_diag, d.S);
    phase_end(p, ENKFMC_PH_DUAL_S, s);
    phase_begin(p, ENKFMC_PH_DUAL_CHOL, s);
    if (dual_chol_tiles_fit(p)) {
      const hipError_t e = launch_dual_chol_tiles(p, d, s);
      if (e != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_dual_chol, dim3(nb), dim3(256), 0, s, d.blocks, d.S, d.status);
    }
    phase_end(p, ENKFMC_PH_DUAL_CHOL, s);
  }
  return hipGetLastError();
}

// X_a = X_b + Z on interior rows.
template <typename TX>
static hipError_t mapback_typed(enkfmc_plan *p, const Dev &d, const TX *Xb, int64_t ld, void *Xa, int32_t out_dtype,
                                hipStream_t s) {
  const int N = p->N;
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

hipError_t launch_mapback(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, void *Xa,
                          int32_t out_dtype, hipStream_t s) {
  if (dtype == ENKFMC_F32) return mapback_typed(p, d, (const float *)Xb, ld, Xa, out_dtype, s);
  return mapback_typed(p, d, (const double *)Xb, ld, Xa, out_dtype, s);
}

template <typename TX>
static hipError_t analysis_typed(enkfmc_plan *p, const Dev &d, const TX *Xb, int64_t ld, const double *Y,
                                 const double *r_diag, void *Xa, int32_t out_dtype, hipStream_t s) {
  const unsigned nb = (unsigned)p->blocks.size();
  const int N = p->N;
  hipError_t e = launch_dual_factor(p, d, r_diag, s);
  if (e != hipSuccess) return e;
  if (p->max_bm > 0) {
    phase_begin(p, ENKFMC_PH_DUAL_Q, s);
    if (solve_S_tiles_fit(p))
      launch_solve_S<TX>(p, d, 0, Xb, ld, Y, d.Q, s);
    else
      hipLaunchKernelGGL(k_dual_Q<TX>, dim3(nb, (N + 63) / 64), dim3(64), 0, s, d.blocks, d.bobs_o, d.bobs_row,
                         d.fit_glob, d.S, Y, Xb, ld, N, d.Q);
    phase_end(p, ENKFMC_PH_DUAL_Q, s);
  }
  e = launch_fwd_sweep(p, d, d.Q, nullptr, d.Z, s);
  if (e != hipSuccess) return e;
  return mapback_typed(p, d, Xb, ld, Xa, out_dtype, s);
}


hipError_t launch_analysis_dual(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld,
                                const double *Y, const double *r_diag, void *Xa, int32_t out_dtype, hipStream_t s) {
  if (dtype == ENKFMC_F32) return analysis_typed(p, d, (const float *)Xb, ld, Y, r_diag, Xa, out_dtype, s);
  return analysis_typed(p, d, (const double *)Xb, ld, Y, r_diag, Xa, out_dtype, s);
}

}  // namespace enkfmc
