// Reverse-mode derivative of fit + local analysis.
//
// Forward, per (sub-domain, variable) block (eq. 11 per sub-domain):
//   A Z = H^T R^-1 Delta,  A = T^T D^-1 T + H^T R^-1 H,  Delta = Y^s - H X_b,
//   X_a = X_b + Z on interior rows;
// per row i of T (eq. 1, ridge lam on the (N-1)-normalised Gram):
//   G beta = c,  G = U_P U_P^T/(N-1) + lam I,  c = U_P u_i/(N-1),
//   eps = u_i - U_P^T beta,  d_i = eps^T eps/(N-1),  T_{i,P} = -beta,
// with u the ensemble anomalies of eq. (5).
//
// Reverse pass, given Gbar = dL/dX_a:
//   Zbar = Gbar on interior rows, 0 on halo rows.
//   W = A^-1 Zbar through the dual form (Woodbury, as eqs. 12-13):
//     V = T^-T Zbar,  P = S^-1 (F^T D V),  W = T^-1 D (V - F P),
//     with F = T^-T H^T and S = R + F^T D F (Cholesky kept by the analysis),
//     since H T^-1 = F^T.
//   Observations:  dlog r_o = (1/r_o) W_j . (Z_j - Delta_o),
//                  dX_b[obs_o] -= W_j / r_o                  (j = local row of o).
//   Factors (Abar = -W Z^T, symmetric part):
//     Dbar_i     = d_i^-2 (T W)_i . (T Z)_i
//     betabar_iq = [(T Z)_i . W_q + (T W)_i . Z_q] / d_i      (q in P(i))
//   Regression of row i, recomputing its Gram and Cholesky:
//     epsbar = 2 Dbar_i eps/(N-1),  b = betabar - U_P epsbar,  s = G^-1 b,
//     lambar_i = -s . beta,  g = U_P^T s,
//     e1_i = eps/(N-1),  e2_i = -(g/(N-1) + epsbar)
//   so that Ubar_q = sum over rows i with q in P(i) of (s_iq e1_i + beta_iq e2_i)
//   and ubar_i gets -e2_i.  Anomalies (eq. 5): dX_b += Ubar - mean_members(Ubar).
// Every sum over sub-domains (overlapping halos) and over observations is a
// gather in a fixed order, so the result is bitwise repeatable.
#include "device.h"

namespace enkfmc {


// Zbar of fit row f: the output gradient of its component if f is the row that
// maps back onto it, else 0.
__device__ inline double zbar_of(const int32_t *fit_glob, const int32_t *interior_src, const double *dXa, int N,
                                 int64_t f, int col) {
  const int g = fit_glob[f];
  return interior_src[g] == f ? dXa[(int64_t)g * N + col] : 0.0;
}

// V = T^-T Zbar, backward over row tiles; one wavefront per (block, 16 member columns).
__global__ __launch_bounds__(64) void k_adj_bwd_sweep(const Block *__restrict__ blocks,
                                                      const int64_t *__restrict__ ct_ptr,
                                                      const int32_t *__restrict__ ct_row,
                                                      const int32_t *__restrict__ ct_slot,
                                                      const int32_t *__restrict__ fit_glob,
                                                      const int32_t *__restrict__ interior_src,
                                                      const double *__restrict__ tiles,
                                                      const double *__restrict__ tinv, const double *__restrict__ dXa,
                                                      int N, double *__restrict__ V) {
  const Block B = blocks[blockIdx.x];
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * blockIdx.y + c;
  const bool colok = colj < N;
  double *Vb = V + B.row0 * N;
  for (int C = B.nrt - 1; C >= 0; --C) {
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * C + 4 * r + q;
      acc[r] = (row < B.n && colok) ? zbar_of(fit_glob, interior_src, dXa, N, B.row0 + row, colj) : 0.0;
    }
    const int64_t s0 = ct_ptr[B.rt0 + C], s1 = ct_ptr[B.rt0 + C + 1];
    for (int64_t t = s0; t < s1; ++t) {
      const int R = ct_row[t];
      const double *Tt = tiles + (int64_t)ct_slot[t] * 256;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int row = 16 * R + 4 * kc + q;
        const double v = (row < B.n && colok) ? Vb[(int64_t)row * N + colj] : 0.0;
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
        if (row < B.n) Vb[(int64_t)row * N + colj] = out[r];
      }
    }
  }
}

// V = T^-T Zbar split by tile distance (as the forward sweep): column tiles
// descend in chunks of D + 1; a far tile T_RC (R - C > D, a suffix of the
// column's ascending list) has R in a later chunk, so the chunk's far sums are
// independent products with V_R from memory, four tiles' loads at a time; the
// near tiles follow from a ring of the last D V tiles in LDS.  One wavefront
// per (block, 16 member columns), XCD-contiguous.
template <int D>
__global__ __launch_bounds__(64) void k_adj_bwd_sweep_near(const Block *__restrict__ blocks, int ng,
                                                           const int64_t *__restrict__ ct_ptr,
                                                           const int32_t *__restrict__ ct_row,
                                                           const int32_t *__restrict__ ct_slot,
                                                           const int32_t *__restrict__ ct_nfar,
                                                           const int32_t *__restrict__ fit_glob,
                                                           const int32_t *__restrict__ interior_src,
                                                           const double *__restrict__ tiles,
                                                           const double *__restrict__ tinv,
                                                           const double *__restrict__ dXa, int N,
                                                           double *__restrict__ V) {
  constexpr int W = D + 1;
  constexpr int kFarBatch = 4;
  __shared__ double ring[D * 256];
  const int64_t lg = xcd_contiguous(blockIdx.x, gridDim.x);
  const Block B = blocks[lg / ng];
  const int cc = (int)(lg % ng);
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * cc + c;
  const bool colok = colj < N;
  double *Vb = V + B.row0 * N;
  const int64_t *cp = ct_ptr + B.rt0;
  for (int C0 = B.nrt - 1; C0 >= 0; C0 -= W) {
    d4 acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int C = C0 - j;
      acc[j] = d4{0.0, 0.0, 0.0, 0.0};
      if (C < 0) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * C + 4 * r + q;
        acc[j][r] = (row < B.n && colok) ? zbar_of(fit_glob, interior_src, dXa, N, B.row0 + row, colj) : 0.0;
      }
      const int64_t tf1 = cp[C + 1], tf0 = tf1 - ct_nfar[B.rt0 + C];
      for (int64_t tb = tf0; tb < tf1; tb += kFarBatch) {
        double ta[kFarBatch][4], vv[kFarBatch][4];
#pragma unroll
        for (int u = 0; u < kFarBatch; ++u) {
          const bool in = tb + u < tf1;
          const int64_t t = in ? tb + u : tf0;
          const int R = ct_row[t];
          const double *Tt = tiles + (int64_t)ct_slot[t] * 256;
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const int row = 16 * R + 4 * kc + q;
            ta[u][kc] = in ? Tt[(4 * kc + q) * 16 + c] : 0.0;   // A: T_RC(4kc + q, c)
            vv[u][kc] = (row < B.n && colok) ? Vb[(int64_t)row * N + colj] : 0.0;   // B: V_R(4kc + q, colj)
          }
        }
#pragma unroll
        for (int u = 0; u < kFarBatch; ++u)
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) acc[j] = mfma64(-ta[u][kc], vv[u][kc], acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int C = C0 - j;
      if (C < 0) break;
      d4 a0 = acc[j], a1 = d4{0.0, 0.0, 0.0, 0.0};
      const int64_t tn0 = cp[C], tn1 = cp[C + 1] - ct_nfar[B.rt0 + C];
#pragma unroll
      for (int u = 0; u < D; ++u) {
        if (tn0 + u >= tn1) break;
        const int R = ct_row[tn0 + u];
        const double *Tt = tiles + (int64_t)ct_slot[tn0 + u] * 256 + q * 16 + c;
        const double *vr = ring + (R % D) * 256 + 16 * q + c;   // B operand: V_R(4kc + q, c)
        a0 = mfma64(-Tt[0], vr[0], a0);
        a1 = mfma64(-Tt[128], vr[128], a1);
        a0 = mfma64(-Tt[64], vr[64], a0);
        a1 = mfma64(-Tt[192], vr[192], a1);
      }
      const d4 sum = a0 + a1;
      const double *Ti = tinv + (B.rt0 + C) * 256 + q * 16 + c;
      d4 out = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) out = mfma64(Ti[64 * kc], sum[kc], out);
      wave_lds_sync();   // every read of the slot's previous tile (V_{C+D}) is done
      double *slot = ring + (C % D) * 256 + 16 * q + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        slot[64 * r] = out[r];
        const int row = 16 * C + 4 * r + q;
        if (colok && row < B.n) Vb[(int64_t)row * N + colj] = out[r];
      }
      wave_lds_sync();
    }
  }
}

// P = F^T D V (ldf x N per block); one wavefront per (block, 16 member columns,
// chunk of up to 8 observation tiles).
__global__ __launch_bounds__(64) void k_adj_ftdv(const Block *__restrict__ blocks, const int32_t *__restrict__ ot_jmax,
                                                 const double *__restrict__ F, const double *__restrict__ dvec,
                                                 const double *__restrict__ V, int N, double *__restrict__ P) {
  constexpr int kMaxTiles = 8;
  const Block B = blocks[blockIdx.x];
  const int TI = B.ldf >> 4;
  const int I0 = kMaxTiles * (int)blockIdx.z;
  if (B.m == 0 || I0 >= TI) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  const int colj = 16 * blockIdx.y + c;
  const bool colok = colj < N;
  const int ldf = B.ldf;
  const double *Fb = F + B.F0;
  const double *Vb = V + B.row0 * N;
  d4 acc[kMaxTiles];
#pragma unroll
  for (int I = 0; I < kMaxTiles; ++I) acc[I] = d4{0.0, 0.0, 0.0, 0.0};
  // the chunk's columns of F vanish below their largest observed row
  int jm = 0;
  for (int i = 0; i < kMaxTiles && I0 + i < TI; ++i) jm = max(jm, ot_jmax[B.ot0 + I0 + i]);
  const int ksteps = (jm >> 2) + 1;
  for (int ks = 0; ks < ksteps; ++ks) {
    const int k = 4 * ks + q;
    const bool in = k < B.n && colok;
    const double b = in ? dvec[B.row0 + k] * Vb[(int64_t)k * N + colj] : 0.0;
    const double *Fk = Fb + (int64_t)k * ldf + c;
#pragma unroll
    for (int i = 0; i < kMaxTiles; ++i)
      if (I0 + i < TI) acc[i] = mfma64(Fk[16 * (I0 + i)], b, acc[i]);
  }
  if (!colok) return;
  double *Pb = P + B.Q0;
#pragma unroll
  for (int i = 0; i < kMaxTiles; ++i) {
    if (I0 + i < TI) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Pb[(int64_t)(16 * (I0 + i) + 4 * r + q) * N + colj] = acc[i][r];
    }
  }
}

// P <- S^-1 P with the Cholesky factor the analysis left in S; one lane per member.
__global__ __launch_bounds__(64) void k_adj_solve_S(const Block *__restrict__ blocks, const double *__restrict__ S,
                                                    int N, double *__restrict__ P) {
  const Block B = blocks[blockIdx.x];
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= N || B.m == 0) return;
  const int m = B.m, lds = B.ldf;
  const double *L = S + B.S0;
  double *x = P + B.Q0;
  chol_solve_col(L, lds, m, x + c, N);
  for (int a = m; a < lds; ++a) x[(int64_t)a * N + c] = 0.0;
}

// Dbar and betabar by 16-row tiles of T.  One workgroup per (block, row tile
// R), one wavefront per member tile g (N <= 16 G).  First TZ_R = Z_R +
// sum_C T_RC Z_C and TW_R likewise (C over the pattern's tiles of R, the
// strictly lower T_RR included), over the wave's 16 members, accumulated
// transposed: with the operands of each v_mfma_f64_16x16x4 swapped, the
// accumulator holds (TZ_R)^T, so lane (q, c) keeps row c of TZ_R and TW_R --
// exactly the A operands the 16 x 16 products below need, so they stay in
// registers (scaled by 1/d_c).
// Dbar_i = (TW)_i . (TZ)_i / d_i^2: each wave sums its members, the partials
// meet in LDS and are added in member-tile order.  Then per tile (R, C) of the
// pattern each wave forms its members' share of (TZ_R/d) W_C^T + (TW_R/d)
// Z_C^T; the shares are added in LDS in member-tile order, and the entries in
// the pattern of T are betabar, written in CSR order.
// Member order: register r of lane (q, c) holds member 16g + 4q + r (the A
// operand of pass 1 takes member 16g + pi(c), pi(4r + q) = 4q + r), and
// k-step kc of pass 1 takes row 4q + kc of the tile.  Every lane then loads
// four consecutive doubles of a row (T_RC in pass 1, W_C and Z_C in pass 2):
// with WIDE (N a multiple of 4, rows 32-byte aligned) as two 16-byte loads,
// which touch half the cache lines of four 8-byte ones spread over 16 rows.
template <int G, bool WIDE>
__global__ __launch_bounds__(64 * G) void k_adj_factor_tiles(const Block *__restrict__ blocks,
                                                             const int64_t *__restrict__ row_ptr,
                                                             const int32_t *__restrict__ col,
                                                             const int64_t *__restrict__ rt_ptr,
                                                             const int32_t *__restrict__ rt_col,
                                                             const int32_t *__restrict__ rt_slot,
                                                             const uint16_t *__restrict__ teoff,
                                                             const double *__restrict__ tiles,
                                                             const double *__restrict__ tdiag,
                                                             const double *__restrict__ dvec,
                                                             const double *__restrict__ Z,
                                                             const double *__restrict__ W, int N, int ntile,
                                                             double *__restrict__ dbar, double *__restrict__ bbar) {
  __shared__ double sred[2][G][16 * 17];   // per-wave 16 x 16 shares, double-buffered over tiles
  __shared__ double sdp[G][16];
  __shared__ int64_t srow[2][16];          // CSR start and end of the tile's rows
  int bi, R;
  block_tile(ntile, bi, R);
  const Block B = blocks[bi];
  if (R >= B.nrt) return;
  const int tid = threadIdx.x, g = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
  const int64_t rt = B.rt0 + R;
  const int64_t t0 = rt_ptr[rt];
  const int nt = (int)(rt_ptr[rt + 1] - t0);
  const double *Zb = Z + B.row0 * N, *Wb = W + B.row0 * N;
  const int rowc = 16 * R + c;                   // the row this lane's accumulators hold
  const double dinv = rowc < B.n ? 1.0 / dvec[B.row0 + rowc] : 0.0;
  if (tid < 16) {
    const int row = 16 * R + tid;
    srow[0][tid] = row < B.n ? row_ptr[B.row0 + row] : 0;
    srow[1][tid] = row < B.n ? row_ptr[B.row0 + row + 1] : 0;
  }
  const int mq = 16 * g + 4 * q;                 // members mq .. mq + 3 of this lane's registers
  // four consecutive doubles of a row at members mq..mq+3 (zero past N or past the block)
  auto row4 = [&](const double *base, int row, bool rin, double (&v)[4]) {
    if constexpr (WIDE) {
      if (rin && mq < N) {
        const d2 *p2 = (const d2 *)(base + (int64_t)row * N + mq);
        const d2 lo = p2[0], hi = p2[1];
        v[0] = lo[0]; v[1] = lo[1]; v[2] = hi[0]; v[3] = hi[1];
      } else {
        v[0] = v[1] = v[2] = v[3] = 0.0;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = rin && mq + r < N ? base[(int64_t)row * N + mq + r] : 0.0;
    }
  };
  d4 az, aw;
  {
    // identity part: (Z_R)^T at lane (q, c), register r: Z[16R + c][16g + 4q + r]
    double zr[4], wr[4];
    row4(Zb, rowc, rowc < B.n, zr);
    row4(Wb, rowc, rowc < B.n, wr);
    az = d4{zr[0], zr[1], zr[2], zr[3]};
    aw = d4{wr[0], wr[1], wr[2], wr[3]};
  }
  const int mp = 16 * g + 4 * (c & 3) + (c >> 2);   // member of this lane's A operands in pass 1
  const bool mpok = mp < N;
  for (int t = 0; t <= nt; ++t) {                // t == nt: the diagonal tile
    const int C = t < nt ? rt_col[t0 + t] : R;
    const double *Tt = t < nt ? tiles + (int64_t)rt_slot[t0 + t] * 256 : tdiag + rt * 256;
    // B operand of k-step kc: T_RC^T[4q + kc][c] = T_RC[c][4q + kc]
    const d2 *t2 = (const d2 *)(Tt + c * 16 + 4 * q);
    const d2 tlo = t2[0], thi = t2[1];
    const double tb[4] = {tlo[0], tlo[1], thi[0], thi[1]};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int zr = 16 * C + 4 * q + kc;          // A operand: Z_C^T[mp][4q + kc]
      const bool in = zr < B.n && mpok;
      az = mfma64(in ? Zb[(int64_t)zr * N + mp] : 0.0, tb[kc], az);
      aw = mfma64(in ? Wb[(int64_t)zr * N + mp] : 0.0, tb[kc], aw);
    }
  }
  double dp = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    dp = fma(az[r], aw[r], dp);
    az[r] *= dinv;
    aw[r] *= dinv;
  }
  dp += __shfl_xor(dp, 16, 64);
  dp += __shfl_xor(dp, 32, 64);
  if (q == 0) sdp[g][c] = dp;
  __syncthreads();
  if (tid < 16 && rowc < B.n) {                  // wave 0, q == 0: row c == tid
    double s = 0.0;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) s += sdp[gg][tid];
    dbar[B.row0 + rowc] = s * dinv * dinv;
  }
  for (int t = 0; t <= nt; ++t) {
    const int C = t < nt ? rt_col[t0 + t] : R;
    const int jr = 16 * C + c;                   // row of W_C, Z_C for the B operand
    double bw[4], bz[4];                         // k-step r: member 16g + 4q + r
    row4(Wb, jr, jr < B.n, bw);
    row4(Zb, jr, jr < B.n, bz);
    d4 o1 = d4{0.0, 0.0, 0.0, 0.0}, o2 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      o1 = mfma64(az[r], bw[r], o1);
      o2 = mfma64(aw[r], bz[r], o2);
    }
    const d4 o = o1 + o2;
    double *so = sred[t & 1][g];
#pragma unroll
    for (int r = 0; r < 4; ++r) so[(4 * r + q) * 17 + c] = o[r];
    __syncthreads();
    // betabar of the entries of tile row i (at most 16, consecutive in CSR
    // order): thread (i, e) takes entry e of row i
    const double(*sb)[16 * 17] = sred[t & 1];
    for (int pr = tid; pr < 256; pr += 64 * G) {
      const int i = pr >> 4, e = pr & 15;
      if (16 * R + i >= B.n) continue;
      const int64_t ka = srow[0][i];
      const int64_t e0 = ka + teoff[16 * (t0 + rt + t) + i];
      const int64_t e1 = t < nt ? ka + teoff[16 * (t0 + rt + t + 1) + i] : srow[1][i];
      const int64_t k = e0 + e;
      if (k < e1) {
        const int j = i * 17 + col[k] - 16 * C;
        double v = 0.0;
#pragma unroll
        for (int gg = 0; gg < G; ++gg) v += sb[gg][j];
        bbar[k] = v;
      }
    }
  }
}

// Solve M x = v in place with the lower Cholesky factor of M in LDS (m x m).
__device__ inline void chol_solve_lds(const double *G, int m, double *v) {
  const int tid = threadIdx.x;
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
}

// Adjoint of each regression: one 256-thread workgroup per fit row.  Reads
// betabar from sb_io and overwrites it with s; writes e1, e2 (n_fit x N) and
// the row's share of dL/dlam.
__global__ __launch_bounds__(256) void k_adj_regress(const Block *__restrict__ blocks,
                                                     const int32_t *__restrict__ fit_glob,
                                                     const int32_t *__restrict__ fit_blk,
                                                     const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, const double *__restrict__ U,
                                                     int ldu, int N, int max_p, double lam,
                                                     const double *__restrict__ tval, const double *__restrict__ dbar,
                                                     double *__restrict__ sb_io, double *__restrict__ e1,
                                                     double *__restrict__ e2, double *__restrict__ lam_row,
                                                     int32_t *status, const int32_t *__restrict__ rows) {
  extern __shared__ double smem[];
  __shared__ int bad;
  const int64_t r = rows ? (int64_t)rows[blockIdx.x] : (int64_t)blockIdx.x;
  const int tid = threadIdx.x;
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const double *u = U + (int64_t)fit_glob[r] * ldu;
  const double mu = lam * (double)(N - 1);
  const double nm1 = (double)(N - 1);
  const bool kform = lam > 0.0 && p >= N;
  const int m = kform ? N : p;
  const int vl = N > max_p ? N : max_p;
  double *G = smem;                         // N*N
  double *v = G + (size_t)N * N;            // vl: right-hand sides / solutions
  double *eps = v + vl;                     // N
  double *ebar = eps + N;                   // N
  double *bb = ebar + N;                    // vl: betabar - U_P epsbar, then s
  double *beta = bb + vl;                   // max_p
  double *red = beta + max_p;               // 8
  int *pidx = (int *)(red + 8);             // max_p
  if (tid == 0) bad = 0;
  for (int k = tid; k < p; k += 256) {
    pidx[k] = fit_glob[B.row0 + col[lo + k]];
    beta[k] = -tval[lo + k];
  }
  __syncthreads();
  const double Db = dbar[r];
  if (p == 0) {
    for (int c = tid; c < N; c += 256) {
      const double ec = 2.0 * Db * u[c] / nm1;
      e1[r * N + c] = u[c] / nm1;
      e2[r * N + c] = -ec;
    }
    if (tid == 0) lam_row[r] = 0.0;
    return;
  }
  // Gram (lower triangle), as the forward fit forms it
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
  } else {
    for (int idx = tid; idx < m * m; idx += 256) {
      const int a = idx / m, b = idx % m;
      if (b > a) continue;
      const double *ua = U + (int64_t)pidx[a] * ldu, *ub = U + (int64_t)pidx[b] * ldu;
      double s = 0.0;
      for (int c = 0; c < N; ++c) s += ua[c] * ub[c];
      G[a * m + b] = s + (a == b ? mu : 0.0);
    }
  }
  __syncthreads();
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
  // residual eps (kernel form: eps = mu w with (U_P^T U_P + mu I) w = u)
  if (kform) {
    for (int c = tid; c < N; c += 256) v[c] = u[c];
    __syncthreads();
    chol_solve_lds(G, m, v);
    for (int c = tid; c < N; c += 256) eps[c] = mu * v[c];
  } else {
    for (int c = tid; c < N; c += 256) {
      double e = u[c];
      for (int a = 0; a < p; ++a) e -= beta[a] * U[(int64_t)pidx[a] * ldu + c];
      eps[c] = e;
    }
  }
  __syncthreads();
  for (int c = tid; c < N; c += 256) ebar[c] = 2.0 * Db * eps[c] / nm1;
  __syncthreads();
  for (int a = tid; a < p; a += 256) {
    const double *ua = U + (int64_t)pidx[a] * ldu;
    double s = sb_io[lo + a];
    for (int c = 0; c < N; ++c) s -= ua[c] * ebar[c];
    bb[a] = s;
  }
  __syncthreads();
  // s = G^-1 bb with G = (U_P U_P^T + mu I)/(N-1)
  if (kform) {
    // (U_P U_P^T + mu I)^-1 = (1/mu) [I - U_P (U_P^T U_P + mu I)^-1 U_P^T]
    for (int c = tid; c < N; c += 256) {
      double t = 0.0;
      for (int a = 0; a < p; ++a) t += U[(int64_t)pidx[a] * ldu + c] * bb[a];
      v[c] = t;
    }
    __syncthreads();
    chol_solve_lds(G, m, v);
    for (int a = tid; a < p; a += 256) {
      const double *ua = U + (int64_t)pidx[a] * ldu;
      double t = 0.0;
      for (int c = 0; c < N; ++c) t += ua[c] * v[c];
      bb[a] = nm1 / mu * (bb[a] - t);
    }
  } else {
    for (int a = tid; a < p; a += 256) v[a] = bb[a];
    __syncthreads();
    chol_solve_lds(G, m, v);
    for (int a = tid; a < p; a += 256) bb[a] = nm1 * v[a];
  }
  __syncthreads();
  double ls = 0.0;
  for (int a = tid; a < p; a += 256) {
    ls -= bb[a] * beta[a];
    sb_io[lo + a] = bb[a];
  }
  ls = block_sum256(ls, red);
  if (tid == 0) lam_row[r] = ls;
  for (int c = tid; c < N; c += 256) {
    double g = 0.0;
    for (int a = 0; a < p; ++a) g += U[(int64_t)pidx[a] * ldu + c] * bb[a];
    e1[r * N + c] = eps[c] / nm1;
    e2[r * N + c] = -(g / nm1 + ebar[c]);
  }
}

size_t adj_regress_lds(const enkfmc_plan *p) {
  const int N = p->N, mp = p->max_p, vl = N > mp ? N : mp;
  return (size_t)N * N * 8 + (size_t)(2 * vl + 2 * N + mp + 8) * 8 + (size_t)mp * 4 + 16;
}

// Ubar of every fit row by 16-row column tiles: for column tile C of a block,
//   Ubar_C = sum_R (S_RC^T E1_R - T_RC^T E2_R) - E2_C
// over the pattern's tiles (R, C), the diagonal tile included (strictly lower
// parts); S holds the rows' s in the pattern of T.  One workgroup per (block,
// column tile), one wavefront per member tile g (N <= 16 G): the members are
// independent columns of the products.  The workgroup assembles each S_RC in
// LDS from the CSR entries (double-buffered over tiles); T_RC comes from the
// dense tiles.
template <int G>
__global__ __launch_bounds__(64 * G) void k_adj_ubar_tiles(const Block *__restrict__ blocks,
                                                           const int64_t *__restrict__ row_ptr,
                                                           const int32_t *__restrict__ col,
                                                           const int64_t *__restrict__ rt_ptr,
                                                           const uint16_t *__restrict__ teoff,
                                                           const int64_t *__restrict__ ct_ptr,
                                                           const int32_t *__restrict__ ct_row,
                                                           const int32_t *__restrict__ ct_slot,
                                                           const double *__restrict__ tiles,
                                                           const double *__restrict__ tdiag,
                                                           const double *__restrict__ sv,
                                                           const double *__restrict__ e1,
                                                           const double *__restrict__ e2, int N, int ntile,
                                                           double *__restrict__ ubar) {
  __shared__ double sS[2][16 * 17];
  int bi, C;
  block_tile(ntile, bi, C);
  const Block B = blocks[bi];
  if (C >= B.nrt) return;
  const int tid = threadIdx.x, g = tid >> 6, lane = tid & 63, q = lane >> 4, c = lane & 15;
  const double *E1 = e1 + B.row0 * N, *E2 = e2 + B.row0 * N;
  const int colj = 16 * g + c;                   // this lane's member
  const bool colok = colj < N;
  d4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * C + 4 * r + q;
    acc[r] = (colok && row < B.n) ? -E2[(int64_t)row * N + colj] : 0.0;
  }
  const int64_t s0 = ct_ptr[B.rt0 + C], s1 = ct_ptr[B.rt0 + C + 1];
  // Per tile (t == s1: the diagonal tile, R = C): the A operands -(T_RC^T)[c][k]
  // (k = 4kc + q), the B operands E1_R, E2_R at rows 16R + k, and the entries
  // of S_RC this thread places: thread (i, e) takes entry e of row i of R
  // within the tile's columns [16C, 16C + 16) (the row's entries of tile (R,
  // C) start at the planned offset and end where the next tile's begin), kept
  // as its slot in the 16 x 17 tile and its value.  Loaded one tile ahead.
  constexpr int kPairs = (256 + 64 * G - 1) / (64 * G);
  auto load = [&](int64_t t, double (&at)[4], double (&b1)[4], double (&b2)[4], int (&js)[kPairs],
                  double (&vs)[kPairs]) {
    const int R = t < s1 ? ct_row[t] : C;
    const double *Tt = t < s1 ? tiles + (int64_t)ct_slot[t] * 256 : tdiag + (B.rt0 + C) * 256;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      at[kc] = -Tt[(4 * kc + q) * 16 + c];
      const int er = 16 * R + 4 * kc + q;
      const bool in = er < B.n && colok;
      b1[kc] = in ? E1[(int64_t)er * N + colj] : 0.0;
      b2[kc] = in ? E2[(int64_t)er * N + colj] : 0.0;
    }
    const int64_t rtR = B.rt0 + R;
#pragma unroll
    for (int it = 0; it < kPairs; ++it) {
      const int pr = tid + 64 * G * it;
      js[it] = -1;
      vs[it] = 0.0;
      const int i = (pr >> 4) & 15, e = pr & 15;
      const int row = 16 * R + i;
      if (pr < 256 && row < B.n) {
        const int64_t ix = 16 * ((t < s1 ? (int64_t)ct_slot[t] : rt_ptr[rtR + 1]) + rtR) + i;
        const int64_t ka = row_ptr[B.row0 + row];
        const int64_t ea = ka + teoff[ix];
        const int64_t eb = t < s1 ? ka + teoff[ix + 16] : row_ptr[B.row0 + row + 1];
        const int64_t k = ea + e;
        if (k < eb) {
          js[it] = i * 17 + col[k] - 16 * C;
          vs[it] = sv[k];
        }
      }
    }
  };
  double at[4], b1[4], b2[4], vs[kPairs];
  int js[kPairs];
  load(s0, at, b1, b2, js, vs);
  for (int64_t t = s0; t <= s1; ++t) {
    double at2[4], b12[4], b22[4], vs2[kPairs];
    int js2[kPairs];
    load(t < s1 ? t + 1 : s1, at2, b12, b22, js2, vs2);
    double *S = sS[(t - s0) & 1];
    for (int e = tid; e < 16 * 17; e += 64 * G) S[e] = 0.0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kPairs; ++it)
      if (js[it] >= 0) S[js[it]] = vs[it];
    __syncthreads();
    // A operands (S_RC^T)[c][k] = S_RC[k][c] with the products
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      acc = mfma64(S[(4 * kc + q) * 17 + c], b1[kc], acc);
      acc = mfma64(at[kc], b2[kc], acc);
    }
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      at[kc] = at2[kc];
      b1[kc] = b12[kc];
      b2[kc] = b22[kc];
    }
#pragma unroll
    for (int it = 0; it < kPairs; ++it) {
      js[it] = js2[it];
      vs[it] = vs2[it];
    }
  }
  if (!colok) return;
  double *Ub = ubar + B.row0 * N;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * C + 4 * r + q;
    if (row < B.n) Ub[(int64_t)row * N + colj] = acc[r];
  }
}

// dX_b of every component: the direct term Gbar plus the anomaly projection of
// Ubar summed over the component's fit rows in sub-domain order.  One
// wavefront per component, N <= 128.
__global__ __launch_bounds__(256) void k_adj_gather(const int64_t *__restrict__ g2f_ptr,
                                                    const int32_t *__restrict__ g2f, const double *__restrict__ ubar,
                                                    const double *__restrict__ dXa, int64_t n, int N,
                                                    double *__restrict__ dXb) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + wave;
  if (j >= n) return;
  double ub[2] = {0.0, 0.0};
  for (int64_t t = g2f_ptr[j]; t < g2f_ptr[j + 1]; ++t) {
    const int64_t f = g2f[t];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cc = lane + 64 * h;
      if (cc < N) ub[h] += ubar[f * N + cc];
    }
  }
  const double mean = wave_sum(ub[0] + ub[1]) / N;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int cc = lane + 64 * h;
    if (cc < N) dXb[j * N + cc] = dXa[j * N + cc] + (ub[h] - mean);
  }
}

// Observation terms: dlog r_o and the innovation's -W_j/r_o on dX_b[obs_o].
// One wavefront per observation; its block entries in block order.
template <typename TX>
__global__ __launch_bounds__(256) void k_adj_obs(const int64_t *__restrict__ o2b_ptr, const int32_t *__restrict__ o2b,
                                                 const int32_t *__restrict__ bobs_fit,
                                                 const int32_t *__restrict__ fit_glob, const double *__restrict__ Z,
                                                 const double *__restrict__ W, const double *__restrict__ Y,
                                                 const TX *__restrict__ Xb, int64_t ld,
                                                 const double *__restrict__ r_diag, int64_t m, int N,
                                                 double *__restrict__ dXb, double *__restrict__ dlogR) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * 4 + wave;
  if (o >= m) return;
  const int64_t e0 = o2b_ptr[o], e1 = o2b_ptr[o + 1];
  const double ro = r_diag[o];
  double dl = 0.0, aw[2] = {0.0, 0.0};
  int64_t g = -1;
  for (int64_t e = e0; e < e1; ++e) {
    const int64_t f = bobs_fit[o2b[e]];
    g = fit_glob[f];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cc = lane + 64 * h;
      if (cc < N) {
        const double w = W[f * N + cc];
        const double delta = Y[o * N + cc] - (double)Xb[g * ld + cc];
        dl += w * (Z[f * N + cc] - delta);
        aw[h] += w;
      }
    }
  }
  dl = wave_sum(dl);
  if (lane == 0) dlogR[o] = dl / ro;
  if (g < 0) return;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int cc = lane + 64 * h;
    if (cc < N) dXb[g * N + cc] -= aw[h] / ro;
  }
}

// dL/dlam = sum of the rows' shares, in a fixed order: workgroup g sums the
// contiguous chunk g (fixed chunking), then one workgroup sums the partials.
__global__ __launch_bounds__(256) void k_adj_lambda(const double *__restrict__ v, int64_t n, int64_t chunk,
                                                    double *__restrict__ out) {
  __shared__ double red[8];
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += v[i];
  s = block_sum256(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// The plain per-row adjoint (one workgroup per regression) over a list of fit
// rows (every row when rows is NULL).
hipError_t launch_adj_regress_plain_rows(enkfmc_plan *p, const Dev &d, double lam, const int32_t *rows,
                                         int64_t nrows, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const size_t lds = adj_regress_lds(p);
  hipError_t e = hipFuncSetAttribute((const void *)k_adj_regress, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adj_regress, dim3((unsigned)nrows), dim3(256), lds, s, d.blocks, d.fit_glob, d.fit_blk,
                     d.row_ptr, d.col, d.U, p->ldu, p->N, p->max_p, lam, d.tval, d.dbar, d.aux3, d.aux1, d.aux2,
                     d.red, d.status, rows);
  return hipGetLastError();
}

template <typename TX>
static hipError_t backward_typed(enkfmc_plan *p, const Dev &d, const TX *Xb, int64_t ld, const double *Y,
                                 const double *r_diag, double lam, const double *dXa, double *dXb, double *dlogR,
                                 double *dridge, hipStream_t s) {
  const unsigned nb = (unsigned)p->blocks.size();
  const int N = p->N;
  const unsigned ct = (unsigned)((N + 15) / 16);
  phase_begin(p, ENKFMC_PH_BACKWARD, s);
  double *V = d.aux1;
  phase_begin(p, ENKFMC_PH_ADJ_SOLVE, s);
#define ADJ_BWD_NEAR(DD)                                                                                         \
  hipLaunchKernelGGL(k_adj_bwd_sweep_near<DD>, dim3(nb * ct), dim3(64), 0, s, d.blocks, (int)ct, d.ct_ptr,        \
                     d.ct_row, d.ct_slot, d.ct_nfar, d.fit_glob, d.interior_src, d.tiles, d.tinv, dXa, N, V)
  if (p->near_d < std::max(1, (int)p->max_rt_back)) {   // far tiles exist: the split sweep
    switch (p->near_d) {
      case 1: ADJ_BWD_NEAR(1); break;
      case 2: ADJ_BWD_NEAR(2); break;
      case 3: ADJ_BWD_NEAR(3); break;
      case 4: ADJ_BWD_NEAR(4); break;
      case 5: ADJ_BWD_NEAR(5); break;
      case 6: ADJ_BWD_NEAR(6); break;
      case 7: ADJ_BWD_NEAR(7); break;
      default: ADJ_BWD_NEAR(8); break;
    }
  } else {
    hipLaunchKernelGGL(k_adj_bwd_sweep, dim3(nb, ct), dim3(64), 0, s, d.blocks, d.ct_ptr, d.ct_row, d.ct_slot,
                       d.fit_glob, d.interior_src, d.tiles, d.tinv, dXa, N, V);
  }
#undef ADJ_BWD_NEAR
  if (p->max_bm > 0) {
    const unsigned ot = (unsigned)((p->max_bm + 15) / 16);
    hipLaunchKernelGGL(k_adj_ftdv, dim3(nb, ct, (ot + 7) / 8), dim3(64), 0, s, d.blocks, d.ot_jmax, d.F, d.dvec,
                       (const double *)V, N, d.P);
    if (solve_S_tiles_fit(p)) {
      const hipError_t es = launch_adj_solve_S_tiles(p, d, d.P, s);
      if (es != hipSuccess) return es;
    } else {
      hipLaunchKernelGGL(k_adj_solve_S, dim3(nb, (N + 63) / 64), dim3(64), 0, s, d.blocks, d.S, N, d.P);
    }
  }
  hipError_t e = launch_fwd_sweep(p, d, d.P, V, d.W, s);
  if (e != hipSuccess) return e;
  phase_end(p, ENKFMC_PH_ADJ_SOLVE, s);
  phase_begin(p, ENKFMC_PH_ADJ_FACTOR, s);
  {
    const int mt = max_block_tiles(p);
#define ADJ_FACTOR(G)                                                                                            \
  do {                                                                                                           \
    if (N % 4 == 0)                                                                                              \
      hipLaunchKernelGGL((k_adj_factor_tiles<G, true>), dim3(nb * (unsigned)mt), dim3(64 * G), 0, s, d.blocks,    \
                         d.row_ptr, d.col, d.rt_ptr, d.rt_col, d.rt_slot, d.tile_eoff, d.tiles, d.tdiag, d.dvec, d.Z, \
                         d.W, N, mt, d.dbar, d.aux3);                                                            \
    else                                                                                                         \
      hipLaunchKernelGGL((k_adj_factor_tiles<G, false>), dim3(nb * (unsigned)mt), dim3(64 * G), 0, s, d.blocks,   \
                         d.row_ptr, d.col, d.rt_ptr, d.rt_col, d.rt_slot, d.tile_eoff, d.tiles, d.tdiag, d.dvec, d.Z, \
                         d.W, N, mt, d.dbar, d.aux3);                                                            \
  } while (0)
    switch ((N + 15) / 16) {   // member tiles kept in registers (N <= 128)
      case 1: ADJ_FACTOR(1); break;
      case 2: ADJ_FACTOR(2); break;
      case 3: ADJ_FACTOR(3); break;
      case 4: ADJ_FACTOR(4); break;
      case 5: ADJ_FACTOR(5); break;
      case 6: ADJ_FACTOR(6); break;
      case 7: ADJ_FACTOR(7); break;
      default: ADJ_FACTOR(8); break;
    }
#undef ADJ_FACTOR
  }
  phase_end(p, ENKFMC_PH_ADJ_FACTOR, s);
  phase_begin(p, ENKFMC_PH_ADJ_REGRESS, s);
  // the form of the preceding fit: the plain per-row adjoint after a plain
  // fit, else the one-wavefront kernels per bucket (their plain bucket again
  // per row)
  e = p->fit_mode == ENKFMC_FIT_PLAIN ? launch_adj_regress_plain_rows(p, d, lam, nullptr, p->n_fit, s)
                                      : launch_adj_regress_batched(p, d, lam, s);
  if (e != hipSuccess) return e;
  phase_end(p, ENKFMC_PH_ADJ_REGRESS, s);
  phase_begin(p, ENKFMC_PH_ADJ_GATHER, s);
  const int mtu = max_block_tiles(p);
#define ADJ_UBAR(G)                                                                                              \
  hipLaunchKernelGGL(k_adj_ubar_tiles<G>, dim3(nb * (unsigned)mtu), dim3(64 * G), 0, s, d.blocks, d.row_ptr, d.col,     \
                     d.rt_ptr, d.tile_eoff, d.ct_ptr, d.ct_row, d.ct_slot, d.tiles, d.tdiag, d.aux3, d.aux1, d.aux2, \
                     N, mtu, d.ubar)
  switch ((N + 15) / 16) {
    case 1: ADJ_UBAR(1); break;
    case 2: ADJ_UBAR(2); break;
    case 3: ADJ_UBAR(3); break;
    case 4: ADJ_UBAR(4); break;
    case 5: ADJ_UBAR(5); break;
    case 6: ADJ_UBAR(6); break;
    case 7: ADJ_UBAR(7); break;
    default: ADJ_UBAR(8); break;
  }
#undef ADJ_UBAR
  hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)((p->n + 3) / 4)), dim3(256), 0, s, d.g2f_ptr, d.g2f, d.ubar, dXa,
                     p->n, N, dXb);
  if (p->m > 0)
    hipLaunchKernelGGL(k_adj_obs<TX>, dim3((unsigned)((p->m + 3) / 4)), dim3(256), 0, s, d.o2b_ptr, d.o2b,
                       d.bobs_fit, d.fit_glob, d.Z, d.W, Y, Xb, ld, r_diag, p->m, N, dXb, dlogR);
  {
    constexpr int kParts = 256;   // partial sums land in dbar, free by now
    const int64_t chunk = (p->n_fit + kParts - 1) / kParts;
    hipLaunchKernelGGL(k_adj_lambda, dim3(kParts), dim3(256), 0, s, (const double *)d.red, p->n_fit, chunk, d.dbar);
    hipLaunchKernelGGL(k_adj_lambda, dim3(1), dim3(256), 0, s, (const double *)d.dbar, (int64_t)kParts,
                       (int64_t)kParts, dridge);
  }
  phase_end(p, ENKFMC_PH_ADJ_GATHER, s);
  phase_end(p, ENKFMC_PH_BACKWARD, s);
  return hipGetLastError();
}

hipError_t launch_backward(enkfmc_plan *p, const Dev &d, const void *Xb, int32_t dtype, int64_t ld, const double *Y,
                           const double *r_diag, double lam, const double *dXa, double *dXb, double *dlogR,
                           double *dridge, hipStream_t s) {
  if (dtype == ENKFMC_F32)
    return backward_typed(p, d, (const float *)Xb, ld, Y, r_diag, lam, dXa, dXb, dlogR, dridge, s);
  return backward_typed(p, d, (const double *)Xb, ld, Y, r_diag, lam, dXa, dXb, dlogR, dridge, s);
}

}  // namespace enkfmc
