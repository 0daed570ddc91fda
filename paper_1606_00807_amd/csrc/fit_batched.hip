// Batched FP64 modified-Cholesky fit (eq. 1 / eq. 8): one 64-lane wavefront
// per regression, everything in registers.
//
// Per regression (p predecessors, N members, ridge mu = lam*(N-1)):
//   m = N (kernel form, p >= N and lam > 0) or m = p (p-form), T = ceil(m/16).
//   1. Gram  G = X^T X (+ mu I) with X = U_P (kernel form, reduction over the
//      p predecessors) or X = U_P^T (p-form, reduction over the N members),
//      accumulated by v_mfma_f64_16x16x4 into the T(T+1)/2 lower 16x16 tiles
//      (those below the diagonal kept transposed).  Rows/columns m..16T-1 are
//      padded with the identity.
//   2. The right-hand side v (v = u, or U_P u accumulated in the same pass) is
//      a bordering row, so factoring [[G, v], [v^T, .]] also yields
//      y = L^-1 v (forward substitution for free).
//   3. Blocked right-looking Cholesky, panel width 16: inside a panel the 16
//      columns are eliminated one at a time in registers (cross-lane moves:
//      DPP row broadcasts and permlane swaps), carrying an identity tile that
//      ends as L_JJ^-T; the tiles below and the trailing tiles then follow by
//      v_mfma_f64_16x16x4 with both operands straight from registers.
//   4. Back substitution L^T x = y, blocked: x_J = L_JJ^-T (y_J - sum L_IJ^T
//      x_I), tile-vector products summed across lanes.
//   5. p-form: beta = x, eps = u - U_P^T beta;
//      kernel form: w = x, beta = U_P w, eps = mu w.   d = eps^T eps/(N-1).
//
// Every (T, form) pair is its own kernel, launched over a precomputed bucket
// of rows, so that each kernel carries only the registers its T needs.  The
// p-form kernels also take the largest member-tile count MT they unroll their
// residual loops for (5 for N <= 80, else 8).  Systems up to T = 5 keep their
// tiles in VGPRs; T = 6..8 run one wavefront per SIMD, with part of the tiles
// held in AGPRs.
//
// The same routine, instantiated with ADJ, is the adjoint of a regression
// (reverse pass of the fit).  Given Dbar = dL/dd and betabar = dL/dbeta of row
// i, with G = U_P U_P^T/(N-1) + lam I and eps = u - U_P^T beta:
//   epsbar = 2 Dbar eps/(N-1),  b = betabar - U_P epsbar,  s = G^-1 b,
//   dL/dlam += -s . beta,  g = U_P^T s,
//   e1 = eps/(N-1),  e2 = -(g/(N-1) + epsbar).
// The right-hand side b (p-form) or U_P^T b (kernel form, where
// (U_P U_P^T + mu I)^-1 = [I - U_P (U_P^T U_P + mu I)^-1 U_P^T]/mu) is formed
// before the Gram, and the same Gram, Cholesky and back substitution follow.
//
// Factor cache (kernel form).  Given a cache slot, the fit stores the factored
// tiles of each kernel-form row (L_IJ^T below the diagonal, L_JJ^-T on it, as
// step 3 leaves them in registers: NT tiles of 64 lanes x 4 doubles, each lane
// its own 32 contiguous bytes).  The kernel-form adjoint then reads them
// instead of recomputing the Gram and the Cholesky (k_adj_kf_pre, _solve,
// _post below): the bordering row's L^-1 v, which the elimination would have
// produced, comes from a blocked forward substitution.
//
// Layout of a v_mfma_f64_16x16x4 accumulator (lane l = 16q + c, register r):
// element (4r + q, c).  A operand: lane l holds A[c][q]; B operand: B[q][c].
#include "device.h"

namespace enkfmc {

constexpr int kMaxT = 8;          // largest tile count handled here (m <= 128, N <= 128)
constexpr int kMaxP = 192;        // largest predecessor count handled here
constexpr int kTileMapFit = 128;  // row-tile distances R - C mapped in LDS (beyond: bisection)

// Dense tiles of T written by the fit itself (when the whole plan runs the
// one-wavefront kernels): a coefficient of row r goes to T_RC (row-major,
// 16 x 16) at (r mod 16, c mod 16), or to the strictly lower diagonal tile.
// The tiles hold zeros off the pattern from the workspace's adoption on, and
// only pattern positions are ever written.
struct TileOut {
  double *tiles, *tdiag;          // NULL tiles: not written here
  const int64_t *rt_ptr;
  const int32_t *rt_col, *rt_slot, *col;
};
// Destination of a coefficient of a row in row tile R of its block, row i of
// the tile, global row tile rt whose tile list starts at t0 (nt tiles), at
// local column colidx: an index into the tiles (>= 0), or -1 - index into
// the diagonal tiles.  tmap holds the slots of the list at R - C.
__device__ __forceinline__ int tile_dest(const TileOut &to, int R, int i, int64_t rt, int64_t t0, int nt,
                                         const int *tmap, int colidx) {
  const int C = colidx >> 4, j = colidx & 15;
  if (C == R) return -1 - (int)(rt * 256 + i * 16 + j);
  int slot;
  if (R - C < kTileMapFit) {
    slot = tmap[R - C];
  } else {   // list position by bisection (column tiles ascending)
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (to.rt_col[t0 + mid] < C) lo = mid + 1; else hi = mid;
    }
    slot = to.rt_slot[t0 + lo];
  }
  return slot * 256 + i * 16 + j;
}
__device__ __forceinline__ void put_tile(double *tiles, double *tdiag, int d, double v) {
  if (d >= 0) tiles[d] = v;
  else tdiag[-1 - d] = v;
}

template <int T>
struct WaveLds {                  // wavefront-private LDS (doubles unless noted)
  int pidx[kMaxP + 8];            // global rows of the predecessors, pad row beyond p
  int tmap[kTileMapFit];          // tile slot of column tile C of the row's row tile, at R - C
  int tdst[kMaxP];                // where coefficient a goes: tiles[d] (d >= 0) or tdiag[-1 - d]
  double vec[16 * (T + 1)];
  double tile[kMaxP + 16 * kMaxT]; // scratch: bordering row, adjoint vectors
};

__device__ inline double readlane_d(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(x) for x > 0: hardware estimate refined by one Newton step.  On
// gfx950 the estimate is within 5.3e-8 relative and one step brings it within
// 4.3e-15 (measured over 4.2M doubles spanning 2^-40..2^40), far inside the
// regressions' error budget.
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double r = fma(-0.5 * x * y, y, 0.5);
  return fma(y, r, y);
}

template <int T>
__device__ __forceinline__ constexpr int tix(int I, int J) { return I * (I + 1) / 2 + J; }

// Data-parallel-primitive move of a double within rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each row of 16 lanes, every lane of the row getting the same value:
// partners i^1 and i^2 inside quads, then the mirrored lane in each half row
// and in the row (each pairs lanes that already hold equal partial sums).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return v;
}

// Lane N of each row of 16 lanes, given to the whole row (DPP row_newbcast,
// one 64-bit move).
template <int N>
__device__ __forceinline__ double row_bcast(double v) {
  return __longlong_as_double(__builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x150 + N, 0xf, 0xf, true));
}

// Sum over the four rows of 16 lanes (lanes c, c + 16, c + 32, c + 48), each
// of them receiving it.  Swapping a register with itself across 16 lanes
// leaves rows (0, 0, 2, 2) and (1, 1, 3, 3), so their sum holds r0 + r1 and
// r2 + r3; the 32-lane swap of that leaves (0, 1, 0, 1) and (2, 3, 2, 3).
__device__ __forceinline__ double pair_sum16(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned l = (unsigned)(b & 0xffffffffll), h = (unsigned)(b >> 32);
  const auto sl = __builtin_amdgcn_permlane16_swap(l, l, false, false);
  const auto sh = __builtin_amdgcn_permlane16_swap(h, h, false, false);
  return __longlong_as_double(((long long)sh[0] << 32) | sl[0]) + __longlong_as_double(((long long)sh[1] << 32) | sl[1]);
}
__device__ __forceinline__ double pair_sum32(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned l = (unsigned)(b & 0xffffffffll), h = (unsigned)(b >> 32);
  const auto sl = __builtin_amdgcn_permlane32_swap(l, l, false, false);
  const auto sh = __builtin_amdgcn_permlane32_swap(h, h, false, false);
  return __longlong_as_double(((long long)sh[0] << 32) | sl[0]) + __longlong_as_double(((long long)sh[1] << 32) | sl[1]);
}
__device__ __forceinline__ double quarter_sum(double v) { return pair_sum32(pair_sum16(v)); }

// Column K of a diagonal tile's elimination (step 3 of fit_row), all in
// registers.  Lane (q, c) holds a[4rr + q][c] in ajj[rr], E[4rr + q][c] in
// eid[rr] and, at q = 0, the bordering row's entry c in ag (left unscaled,
// like the columns).  a[i][K] for the
// lane's rows comes from lane (q, K) of its own row of 16; a[c][K] is taken as
// a[K][c] (lane (K mod 4, c), register K / 4), which the symmetric updates of
// the columns right of K keep equal to it up to rounding.  piv enters as the
// pivot of column K and leaves as that of column K + 1 (a look-ahead on
// a[K+1][K] and a[K+1][K+1] only); 1/sqrt(piv) is kept by lane c = K.
template <int K>
__device__ __forceinline__ void elim_col(const int c, d4 &ajj, d4 &eid, double &ag,
                                         double &piv, double &myinv) {
  const double inv = rsqrt_nr(piv);
  if (c == K) myinv = inv;
  const double ab = row_bcast<K>(ag) * inv;    // scaled bordering entry K (at q = 0)
  if constexpr (K + 1 < 16) {
    constexpr int q1 = (K + 1) & 3, r1 = (K + 1) >> 2;
    const double lnext = readlane_d(ajj[r1], 16 * q1 + K) * inv;
    const double anext = readlane_d(ajj[r1], 16 * q1 + K + 1);
    piv = fma(-lnext, lnext, anext);
  }
  const double colv = quarter_bcast<K & 3>(ajj[K >> 2]);
  const double cv1 = c > K ? colv * inv : 0.0;   // L[c][K]
  const double cv2 = cv1 * inv;
  // Registers whose rows are all <= K are skipped: those rows of the tile
  // are not read again (row K was read above, as the column).  E's column K
  // is zero below row K, so E's registers whose rows all exceed K would not
  // change.
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
    if (4 * rr + 3 > K) ajj[rr] = fma(-row_bcast<K>(ajj[rr]), cv2, ajj[rr]);
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
    if (4 * rr <= K) eid[rr] = fma(-row_bcast<K>(eid[rr]), cv2, eid[rr]);
  ag = fma(-ab, cv1, ag);   // entries c <= K stay as they are (cv1 = 0)
}

// Columns K..kend-1 (kend <= 16: the tile's columns that belong to the
// system; those past it are padding, coupled to nothing, and are left
// alone, their 1/L_cc staying 0); false at the first pivot that is not
// positive (or NaN).
template <int K>
__device__ __forceinline__ bool elim_cols(const int c, d4 &ajj, d4 &eid, double &ag,
                                          double &piv, double &myinv, const int kend) {
  if (K >= kend) return true;
  if (!(piv > 0.0)) return false;
  elim_col<K>(c, ajj, eid, ag, piv, myinv);
  if constexpr (K + 1 < 16) return elim_cols<K + 1>(c, ajj, eid, ag, piv, myinv, kend);
  return true;
}

// Four 16-lane sums at once: on return lanes 4u..4u+3 of each row of 16 hold
// the row's sum of v_u.  The row mirror pairs lane i with 15 - i: the low half
// keeps v0, v1 and the high half v2, v3, each adding its partner's.  The half
// mirror (i with 7 - i) halves that again, leaving v_u in quad u summed over
// four lanes; two quad exchanges finish each sum.
__device__ __forceinline__ double row16_sum4(const double v0, const double v1, const double v2, const double v3,
                                             const int c) {
  const bool lo8 = c < 8;
  const double r0 = (lo8 ? v0 : v2) + dpp_d<0x140>(lo8 ? v2 : v0);   // row_mirror
  const double r1 = (lo8 ? v1 : v3) + dpp_d<0x140>(lo8 ? v3 : v1);
  const bool lo4 = (c & 7) < 4;
  double s = (lo4 ? r0 : r1) + dpp_d<0x141>(lo4 ? r1 : r0);         // row_half_mirror
  s += dpp_d<0xB1>(s);                                                 // quad_perm [1,0,3,2]
  s += dpp_d<0x4E>(s);                                                 // quad_perm [2,3,0,1]
  return s;
}

// Arrays of the adjoint pass.
struct AdjIO {
  const double *dbar;   // dL/dd per fit row
  double *sb;           // per CSR entry: betabar on entry, s on exit
  double *e1, *e2;      // n_fit x N
  double *lam_row;      // per fit row: its share of dL/dlam
  double *ebl;          // wavefront LDS (kMaxP + 8): epsbar (p-form) or b (kernel form) of the row
};

// Adjoint pre-pass of a kernel-form row r, before its Gram.  In the kernel
// form the forward solve gave eps = mu w and beta = U_P w for the solution w
// of (U_P^T U_P + mu I) w = u, so U_P eps = mu beta and
//   b = betabar - U_P epsbar = betabar - (2 Dbar mu/(N-1)) beta
// needs no pass over U_P.  This leaves beta and b in LDS (zero past p) for
// the Gram loop, which sums eps = u - U_P^T beta and U_P^T b from its own
// fragments, and b in sb for the post-pass.
template <int T>
__device__ __forceinline__ void adj_pre_kf(const int lane, const int64_t r, const int p, const int N,
                                           const double mu, WaveLds<T> &L, const double *__restrict__ tval,
                                           const int64_t lo, const AdjIO &adj) {
  const double coef = 2.0 * adj.dbar[r] * mu / (double)(N - 1);
  double *bl = L.tile;             // beta
  double *bv = adj.ebl;            // b
  for (int a = lane; a < kMaxP + 8; a += 64) {
    const double beta = a < p ? -tval[lo + a] : 0.0;
    const double b = a < p ? fma(-coef, beta, adj.sb[lo + a]) : 0.0;
    if (a < kMaxP) bl[a] = beta;
    bv[a] = b;
    if (a < p) adj.sb[lo + a] = b;
  }
  wave_lds_sync();
}

// Back substitution L^T x = y with the factored tiles in registers (step 4
// of fit_row): y enters as the bordering row (entry 16J + c at lane (0, c)
// in yr[J]) and x leaves in y[] (LDS, natural order).  Panel by panel from
// the last: t = y_J - sum_{I>J} L_IJ^T x_I, then x_J = L_JJ^-T t.  Lane (q,
// c) holds L_IJ^T[4rr + q][c] and L_JJ^-T[4rr + q][c] in register rr, so
// both products multiply by the vector's entry c and sum over the row of 16
// lanes; the four sums of a row go in one exchange (row16_sum4), which leaves
// entry 4(c/4) + q in lane (q, c).
// Blocked Cholesky of a symmetric matrix of T 16 x 16 tiles held in
// registers (step 3 of fit_row), of which the first m rows and columns are
// the system and the rest (past m, in the last tile) an identity padding.  Lane (q, c) holds, in register rr of
// acc[tix(I, J)] (I >= J), element (4rr + q, c) of A_IJ^T.  Per panel J the
// 16 columns of the diagonal tile are eliminated one at a time, carrying an
// identity tile E along as extra rows, so that E ends as L_JJ^-T; the tiles
// below then follow as L_IJ = A_IJ L_JJ^-T by MFMA, and the trailing tiles
// take their updates.  Each column's values reach the other lanes by
// cross-lane moves (elim_col).  Columns stay unscaled during the elimination:
// the update uses a[i][k] a[j][k] / piv_k, and at the end each column c is
// scaled once by its 1/L_cc, which also turns its final pivot into L_cc.
// On return acc[tix(I, J)] holds L_IJ^T below the diagonal and L_JJ^-T on it,
// with zeros in the padding's columns of L_JJ^-T (the padding is not
// eliminated), so that solves with these tiles leave zeros there.
// BORDER: a bordering row (entry 16J + c at lane (0, c) of augv[J]) is
// eliminated along and leaves as L^-1 of it; tba is 16 doubles of LDS for it.
// diag_out(J, L_JJ) receives each diagonal tile of the factor as its panel
// is done (element (4rr + q, c) in register rr; only entries with
// 4rr + q >= c are meaningful).  False at the first pivot that is not
// positive (or NaN).
struct NoDiagOut {
  __device__ void operator()(int, const d4 &) const {}
};
template <int T, bool BORDER, typename DiagOut>
__device__ __forceinline__ bool chol_tiles(const int q, const int c, const int m, d4 (&acc)[T * (T + 1) / 2],
                                           double (&augv)[T], double *tba, const DiagOut &diag_out) {
#pragma unroll
  for (int J = 0; J < T; ++J) {
    const bool below = J + 1 < T;
    d4 eid;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) eid[rr] = (4 * rr + q == c) ? 1.0 : 0.0;
    // pivot of the panel's first column (after the trailing updates)
    double piv = readlane_d(acc[tix<T>(J, J)][0], 0);
    double myinv = 0.0;
    // only the last tile can hold padding (T = ceil(m / 16))
    const int kend = J + 1 < T ? 16 : m - 16 * J;
    if (!elim_cols<0>(c, acc[tix<T>(J, J)], eid, augv[J], piv, myinv, kend)) return false;
    if constexpr (BORDER) augv[J] *= myinv;
    diag_out(J, acc[tix<T>(J, J)] * myinv);
    eid *= myinv;   // L_JJ^-T; the accumulator layout is the B operand layout
    // L_JJ itself is not needed again: its slot keeps L_JJ^-T
    acc[tix<T>(J, J)] = eid;
    if (below) {
      // L_IJ^T = L_JJ^-1 A_IJ^T: E's registers as the A operand give E^T =
      // L_JJ^-1, and the stored A_IJ^T is the B operand of its own registers.
#pragma unroll
      for (int I = J + 1; I < T; ++I) {
        d4 a = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) a = mfma64(eid[kc], acc[tix<T>(I, J)][kc], a);
        acc[tix<T>(I, J)] = a;
      }
      // Trailing update, kept transposed: A_{I,I2}^T -= L_{I2,J} L_{I,J}^T, the
      // A operand from the registers of L_{I2,J}^T (negated once) and the B
      // operand those of L_{I,J}^T.  The bordering row enters as row 0 of an A
      // operand, through LDS.
      if constexpr (BORDER) {
        if (q == 0) tba[c] = augv[J];
        wave_lds_sync();
      }
#pragma unroll
      for (int I2 = J + 1; I2 < T; ++I2) {
        const d4 ny = -acc[tix<T>(I2, J)];
#pragma unroll
        for (int I = I2; I < T; ++I) {
          d4 a = acc[tix<T>(I, I2)];
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) a = mfma64(ny[kc], acc[tix<T>(I, J)][kc], a);
          acc[tix<T>(I, I2)] = a;
        }
        if constexpr (BORDER) {
          d4 a = d4{augv[I2], 0.0, 0.0, 0.0};
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const double tv = tba[4 * kc + q];   // read by every lane, used at c = 0
            a = mfma64(c == 0 ? tv : 0.0, ny[kc], a);
          }
          augv[I2] = a[0];
        }
      }
      if constexpr (BORDER) wave_lds_sync();
    }
  }
  return true;
}

template <int T>
__device__ __forceinline__ void back_subst(const int q, const int c, const d4 (&acc)[T * (T + 1) / 2],
                                           const double (&yr)[T], double *y) {
  if (q == 0) {
#pragma unroll
    for (int J = 0; J < T; ++J) y[16 * J + c] = yr[J];
  }
  wave_lds_sync();
  const int jq = 4 * (c >> 2) + q;   // the entry this lane ends up holding
#pragma unroll
  for (int J = T - 1; J >= 0; --J) {
    double t = y[16 * J + jq];
    if (J + 1 < T) {
      double sr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int I = J + 1; I < T; ++I) {
        const double xc = y[16 * I + c];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) sr[rr] = fma(acc[tix<T>(I, J)][rr], xc, sr[rr]);
      }
      t -= row16_sum4(sr[0], sr[1], sr[2], sr[3], c);
    }
    wave_lds_sync();
    if ((c & 3) == 0) y[16 * J + jq] = t;
    wave_lds_sync();
    const double tc = y[16 * J + c];
    double xr[4];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) xr[rr] = acc[tix<T>(J, J)][rr] * tc;
    const double x = row16_sum4(xr[0], xr[1], xr[2], xr[3], c);
    wave_lds_sync();
    if ((c & 3) == 0) y[16 * J + jq] = x;   // x_J overwrites t
    wave_lds_sync();
  }
}

// Forward substitution y = L^-1 v with the factored tiles in registers (what
// the elimination of step 3 forms as its bordering row).  v enters at lane (0,
// c) of vr[J] (entry 16J + c), y leaves the same way and in y[] (LDS, natural
// order); t[] is 16 doubles of LDS scratch.  Lane (q, c) holds L_JI^T[4rr +
// q][c] = L_JI[c][4rr + q] (I < J) and L_JJ^-T[4rr + q][c] = L_JJ^-1[c][4rr
// + q] in register rr, so each tile-vector product is a sum over the lane's
// registers and then over the four rows of 16 lanes, which leaves entry c in
// every lane.  Block J: t_J = v_J - sum_{I<J} L_JI y_I, y_J = L_JJ^-1 t_J.
template <int T>
__device__ __forceinline__ void fwd_subst(const int q, const int c, const d4 (&acc)[T * (T + 1) / 2],
                                          double (&vr)[T], double *y, double *t) {
#pragma unroll
  for (int J = 0; J < T; ++J) {
    double sp = 0.0;
#pragma unroll
    for (int I = 0; I < J; ++I)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) sp = fma(acc[tix<T>(J, I)][rr], y[16 * I + 4 * rr + q], sp);
    const double tj = quarter_bcast<0>(vr[J]) - quarter_sum(sp);
    if (q == 0) t[c] = tj;
    wave_lds_sync();
    double sy = 0.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) sy = fma(acc[tix<T>(J, J)][rr], t[4 * rr + q], sy);
    const double yj = quarter_sum(sy);
    if (q == 0) y[16 * J + c] = yj;
    vr[J] = q == 0 ? yj : 0.0;
    wave_lds_sync();
  }
}

template <int T, bool KF, int MT, bool ADJ = false>
__device__ __forceinline__ void fit_row(const int lane, const int64_t r, const int p, const int N, const double mu,
                                        const double *__restrict__ U, const int ldu, const int uoff, WaveLds<T> &L,
                                        double *__restrict__ tval, const int64_t lo, double *__restrict__ dvec,
                                        int32_t *status, const AdjIO &adj, double *__restrict__ fc = nullptr,
                                        double *__restrict__ ttiles = nullptr, double *__restrict__ tdiag = nullptr) {
  constexpr int NT = T * (T + 1) / 2;
  const int q = lane >> 4, c = lane & 15;
  const int m = KF ? N : p;
  double augv[T];   // bordering row: element 16J + c at lane (q = 0, c)
  // kernel form: eps, epsbar and b in passes of their own; the p-form forms
  // them inside its Gram loop below
  if constexpr (ADJ && KF) adj_pre_kf<T>(lane, r, p, N, mu, L, tval, lo, adj);
  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  // ---- 1. Gram (+ right-hand side) -----------------------------------------
  // Tile (I, J), I > J, is kept transposed: acc[tix(I, J)] holds A_IJ^T (the
  // operands of its products swapped), so that the factorisation below needs
  // no transposes.
  // pidx[k] for k >= p names the all-zero pad row of U, so padded fragments
  // load zeros; the loads of step ks+1 are issued before the MFMAs of ks.
  if (KF) {
    // Pairs of k-steps and no exit inside the loop body: with an exit between
    // the two halves the compiler copied every accumulator on each trip and
    // dropped the prefetch.  An odd last step runs after the loop from the
    // last prefetch; the prefetch one step past the end reads pad entries
    // (pidx holds kMaxP + 8 entries, 4 * 32 + 3 < kMaxP + 8).
    const int ksn = (p + 3) >> 2;   // k-steps with at least one predecessor
    const int kse = ksn & ~1;        // done in pairs; an odd last step follows the loop
    double fa[T], fb[T];
    // adjoint: lane (q, c) also sums beta_a U[P_a][k] and b_a U[P_a][k] over
    // its predecessors a = 4ks + q for members k = 16I + c (eps and U_P^T b),
    // VALU work that runs beside the Gram's products
    double ea[T], ta[T];
    const double *blp = L.tile, *bvp = adj.ebl;
    if constexpr (ADJ) {
#pragma unroll
      for (int I = 0; I < T; ++I) ea[I] = ta[I] = 0.0;
    }
    {
      const int off = L.pidx[q] * ldu + c;
#pragma unroll
      for (int I = 0; I < T; ++I) fa[I] = U[off + 16 * I];
    }
    for (int ks = 0; ks < kse; ks += 2) {
      const int offb = L.pidx[4 * ks + 4 + q] * ldu + c;
#pragma unroll
      for (int I = 0; I < T; ++I) fb[I] = U[offb + 16 * I];
      __builtin_amdgcn_sched_barrier(0);   // keep each half's loads ahead of the other half's products
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(fa[J], fa[I], acc[tix<T>(I, J)]);
      if constexpr (ADJ) {
        const double bb = blp[4 * ks + q], bw = bvp[4 * ks + q];
#pragma unroll
        for (int I = 0; I < T; ++I) {
          ea[I] = fma(bb, fa[I], ea[I]);
          ta[I] = fma(bw, fa[I], ta[I]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      const int offa = L.pidx[4 * ks + 8 + q] * ldu + c;
#pragma unroll
      for (int I = 0; I < T; ++I) fa[I] = U[offa + 16 * I];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(fb[J], fb[I], acc[tix<T>(I, J)]);
      if constexpr (ADJ) {
        const double bb = blp[4 * ks + 4 + q], bw = bvp[4 * ks + 4 + q];
#pragma unroll
        for (int I = 0; I < T; ++I) {
          ea[I] = fma(bb, fb[I], ea[I]);
          ta[I] = fma(bw, fb[I], ta[I]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (ksn & 1) {   // the last prefetch holds k-step ksn - 1
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(fa[J], fa[I], acc[tix<T>(I, J)]);
      if constexpr (ADJ) {
        const double bb = blp[4 * kse + q], bw = bvp[4 * kse + q];
#pragma unroll
        for (int I = 0; I < T; ++I) {
          ea[I] = fma(bb, fa[I], ea[I]);
          ta[I] = fma(bw, fa[I], ta[I]);
        }
      }
    }
    if constexpr (ADJ) {
      // eps_k = u_k - (U_P^T beta)_k, epsbar = 2 Dbar eps/(N-1): e1 = eps/(N-1)
      // and e2 = epsbar for the post-pass; the bordering row is U_P^T b
      const double nm1 = (double)(N - 1);
      const double Db = adj.dbar[r];
#pragma unroll
      for (int I = 0; I < T; ++I) {
        const double es = quarter_sum(ea[I]);
        const double tb = quarter_sum(ta[I]);
        const int k = 16 * I + c;
        const bool ok = k < N;
        const double eps = ok ? U[uoff + k] - es : 0.0;
        if (q == 0 && ok) {
          adj.e1[r * N + k] = eps / nm1;
          adj.e2[r * N + k] = 2.0 * Db * eps / nm1;
        }
        augv[I] = (q == 0 && ok) ? tb : 0.0;
      }
    }
    if constexpr (!ADJ) {
#pragma unroll
      for (int J = 0; J < T; ++J) {
        const int idx = 16 * J + c;
        const double v = U[uoff + idx];
        augv[J] = (idx < N && q == 0) ? v : 0.0;
      }
    }
  } else {
    // lane (q, c) also sums u_k U[P_{16I+c}][k] over the members it loads.
    // (Single-buffered: a double-buffered form of this loop was miscompiled,
    // its live MFMA accumulators being reused as load destinations.)
    const int ksteps = (N + 3) >> 2;
    int base[T];
#pragma unroll
    for (int I = 0; I < T; ++I) base[I] = L.pidx[16 * I + c] * ldu + q;
    double vp[T];
#pragma unroll
    for (int I = 0; I < T; ++I) vp[I] = 0.0;
    // adjoint: lane (q, c) holds beta of predecessor 16I + c; at member
    // k = 4ks + q the 16 lanes of a quarter sum beta_a U[P_a][k], giving
    // eps_k = u_k - U_P^T beta and epsbar_k = 2 Dbar eps_k / (N-1), and vp[I]
    // gathers sum_k U[P_{16I+c}][k] epsbar_k for b = betabar - U_P epsbar
    double bet[T];
    double Db = 0.0;
    if constexpr (ADJ) {
#pragma unroll
      for (int I = 0; I < T; ++I) bet[I] = 16 * I + c < p ? -tval[lo + 16 * I + c] : 0.0;
      Db = adj.dbar[r];
    }
    if constexpr (!ADJ) {
      // One 16-byte load per tile brings members 8ks + 2q and 8ks + 2q + 1;
      // they form two consecutive k-steps of the product (the sum over
      // members does not depend on which k-step takes which member).
      // 8 * ks2 <= ldu, whose columns past N are zero.
      const int ks2 = (N + 7) >> 3;
      for (int ks = 0; ks < ks2; ++ks) {
        double2 f[T];
#pragma unroll
        for (int I = 0; I < T; ++I) f[I] = *(const double2 *)&U[base[I] + q + 8 * ks];
        const double2 uk = *(const double2 *)&U[uoff + 2 * q + 8 * ks];
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
          for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(f[J].x, f[I].x, acc[tix<T>(I, J)]);
#pragma unroll
        for (int I = 0; I < T; ++I) {
#pragma unroll
          for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(f[J].y, f[I].y, acc[tix<T>(I, J)]);
          vp[I] = fma(f[I].x, uk.x, vp[I]);
          vp[I] = fma(f[I].y, uk.y, vp[I]);
        }
      }
    } else {
      // one 16-byte load per tile brings members 8ks + 2q and 8ks + 2q + 1,
      // two k-steps of the products (as in the fit above); 8 * ks2 <= ldu
      const int ks2 = (N + 7) >> 3;
      const double nm1 = (double)(N - 1);
      for (int ks = 0; ks < ks2; ++ks) {
        double2 f[T];
#pragma unroll
        for (int I = 0; I < T; ++I) f[I] = *(const double2 *)&U[base[I] + q + 8 * ks];
        const double2 uk = *(const double2 *)&U[uoff + 2 * q + 8 * ks];
        double es0 = 0.0, es1 = 0.0;
#pragma unroll
        for (int I = 0; I < T; ++I) {
#pragma unroll
          for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(f[J].x, f[I].x, acc[tix<T>(I, J)]);
          es0 = fma(bet[I], f[I].x, es0);
        }
#pragma unroll
        for (int I = 0; I < T; ++I) {
#pragma unroll
          for (int J = 0; J <= I; ++J) acc[tix<T>(I, J)] = mfma64(f[J].y, f[I].y, acc[tix<T>(I, J)]);
          es1 = fma(bet[I], f[I].y, es1);
        }
        es0 = row16_sum(es0);
        es1 = row16_sum(es1);
        const int k0 = 8 * ks + 2 * q, k1 = k0 + 1;
        const double eps0 = k0 < N ? uk.x - es0 : 0.0, eps1 = k1 < N ? uk.y - es1 : 0.0;
        const double eb0 = 2.0 * Db * eps0 / nm1, eb1 = 2.0 * Db * eps1 / nm1;
        if (c == 0 && k0 < N) {
          adj.e1[r * N + k0] = eps0 / nm1;
          adj.ebl[k0] = eb0;
        }
        if (c == 0 && k1 < N) {
          adj.e1[r * N + k1] = eps1 / nm1;
          adj.ebl[k1] = eb1;
        }
#pragma unroll
        for (int I = 0; I < T; ++I) vp[I] = fma(f[I].y, eb1, fma(f[I].x, eb0, vp[I]));
      }
    }
    if constexpr (ADJ) {
#pragma unroll
      for (int I = 0; I < T; ++I) {
        vp[I] = quarter_sum(vp[I]);
        const int a = 16 * I + c;
        augv[I] = (a < p && q == 0) ? adj.sb[lo + a] - vp[I] : 0.0;   // b_a
      }
    } else {
#pragma unroll
      for (int I = 0; I < T; ++I) {
        vp[I] = quarter_sum(vp[I]);
        augv[I] = (16 * I + c < m && q == 0) ? vp[I] : 0.0;
      }
    }
  }
  // ridge on the diagonal, identity on the padding: the padded rows and
  // columns of the Gram are exactly zero, so adding 1 there gives it
  d4 dmask;   // 1 where register rr holds a diagonal entry
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) dmask[rr] = (4 * rr + q == c) ? 1.0 : 0.0;
#pragma unroll
  for (int J = 0; J < T; ++J) {
    const double dv = 16 * J + c < m ? mu : 1.0;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[tix<T>(J, J)][rr] = fma(dmask[rr], dv, acc[tix<T>(J, J)][rr]);
  }

  // ---- 3. blocked Cholesky of the bordered matrix -------------------------
  if (!chol_tiles<T, true>(q, c, m, acc, augv, L.tile, NoDiagOut{})) {
    if (lane == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }

  // the factored tiles to the cache slot (fit with a factor cache)
  if constexpr (!ADJ) {
    if (fc) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double2 *dst = (double2 *)(fc + (size_t)(64 * t + lane) * 4);
        dst[0] = double2{acc[t][0], acc[t][1]};
        dst[1] = double2{acc[t][2], acc[t][3]};
      }
    }
  }

  // ---- 4. back substitution L^T x = y (y = the factored bordering row) ----
  double *y = L.vec;   // x, natural order
  back_subst<T>(q, c, acc, augv, y);

  if constexpr (!ADJ) {
  // ---- 5. coefficients and residual variance --------------------------------
  // x (= w or beta) is zero beyond m, so the padded terms below vanish.
  double ss = 0.0;
  if (KF) {
    // beta_a = sum_k U[P_a][k] w_k: lane (q, c) loads members 16I + c of
    // predecessor 4ks + q (the Gram's coalesced fragments); the 16 lanes of
    // each quarter then add their partial sums.
    // Four k-steps per trip, their loads issued together (the steps are
    // independent; one at a time each waited for its own loads).  Steps past
    // the last read the zero pad row (pidx holds kMaxP + 8 entries).
    double wv[T];
#pragma unroll
    for (int I = 0; I < T; ++I) wv[I] = y[16 * I + c];
    const int ks4 = (((p + 3) >> 2) + 3) & ~3;
    for (int ks0 = 0; ks0 < ks4; ks0 += 4) {
      double f[4][T];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int off = L.pidx[4 * (ks0 + u) + q] * ldu + c;
#pragma unroll
        for (int I = 0; I < T; ++I) f[u][I] = U[off + 16 * I];
      }
      double bu[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bu[u] = 0.0;
#pragma unroll
        for (int I = 0; I < T; ++I) bu[u] = fma(f[u][I], wv[I], bu[u]);
      }
      // lanes 4u..4u+3 get beta of predecessor 4(ks0 + u) + q
      const double b = row16_sum4(bu[0], bu[1], bu[2], bu[3], c);
      const int a = 4 * (ks0 + (c >> 2)) + q;
      if ((c & 3) == 0 && a < p) {
        tval[lo + a] = -b;
        if (ttiles) put_tile(ttiles, tdiag, L.tdst[a], -b);
      }
    }
    if (q == 0) {
#pragma unroll
      for (int I = 0; I < T; ++I) {
        const double e = mu * y[16 * I + c];
        ss += e * e;
      }
    }
  } else {
    // eps_k = u_k - sum_a beta_a U[P_a][k]: lane (q, c) takes member 16I + c and
    // predecessors a = q mod 4; the four partial sums are then added across q.
    for (int a = lane; a < p; a += 64) {
      tval[lo + a] = -y[a];
      if (ttiles) put_tile(ttiles, tdiag, L.tdst[a], -y[a]);
    }
    // one pointer per predecessor; the member tiles then differ by constant
    // offsets (the loop over them is unrolled, N <= 16 MT)
    double bq[4 * T];
    const double *up[4 * T];
#pragma unroll
    for (int j = 0; j < 4 * T; ++j) {
      bq[j] = y[4 * j + q];
      up[j] = U + ((int64_t)L.pidx[4 * j + q] * ldu + c);
    }
#pragma unroll
    for (int I = 0; I < MT; ++I) {
      if (16 * I >= N) break;
      double e = 0.0;
#pragma unroll
      for (int j = 0; j < 4 * T; ++j) e = fma(bq[j], up[j][16 * I], e);
      e = quarter_sum(e);
      if (q == 0 && 16 * I + c < N) {
        const double eps = U[uoff + 16 * I + c] - e;
        ss += eps * eps;
      }
    }
  }
  ss = wave_sum(ss);
  if (lane == 0) {
    const double dd = ss / (N - 1);
    dvec[r] = dd;
    if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
  }
  } else {
    // ---- 5'. adjoint: s, dL/dlam, e2 ------------------------------------------
    const double nm1 = (double)(N - 1);
    double ls = 0.0;
    if (KF) {
      // s_a = (N-1)/mu (b_a - sum_k U[P_a][k] x_k) and g = U_P^T s from the same
      // fragments (lanes as for beta above); e2 = -(g/(N-1) + epsbar)
      double wv[T], gacc[T];
#pragma unroll
      for (int I = 0; I < T; ++I) {
        wv[I] = y[16 * I + c];
        gacc[I] = 0.0;
      }
      // four k-steps of fragment loads at a time (pad row past the last)
      constexpr int kB = 4;
      const int ksb = (((p + 3) >> 2) + kB - 1) & ~(kB - 1);
      for (int ks0 = 0; ks0 < ksb; ks0 += kB) {
        double f[kB][T];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int off = L.pidx[4 * (ks0 + u) + q] * ldu + c;
#pragma unroll
          for (int I = 0; I < T; ++I) f[u][I] = U[off + 16 * I];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int a = 4 * (ks0 + u) + q;
          double b = 0.0;
#pragma unroll
          for (int I = 0; I < T; ++I) b = fma(f[u][I], wv[I], b);
          b = row16_sum(b);
          const double sv = a < p ? (nm1 / mu) * (adj.sb[lo + a] - b) : 0.0;
          if (c == 0 && a < p) {
            adj.sb[lo + a] = sv;
            ls = fma(sv, tval[lo + a], ls);
          }
#pragma unroll
          for (int I = 0; I < T; ++I) gacc[I] = fma(f[u][I], sv, gacc[I]);
        }
      }
#pragma unroll
      for (int I = 0; I < T; ++I) {
        double e = gacc[I];
        e = quarter_sum(e);
        const int k = 16 * I + c;
        if (q == 0 && k < N) adj.e2[r * N + k] = -(e / nm1 + adj.e2[r * N + k]);
      }
    } else {
      // s overwrites betabar in sb (betabar was read into the right-hand side
      // before the factorisation)
      double *sl = L.tile;     // s (kMaxP entries)
      for (int ks = 0; 4 * ks < p; ++ks) {
        const int a = 4 * ks + q;
        if (c == 0 && a < p) {
          const double sv = nm1 * y[a];
          sl[a] = sv;
          adj.sb[lo + a] = sv;
          ls = fma(sv, tval[lo + a], ls);
        }
      }
      // s is zero past p, up to the last k-step batch
      const int ks4 = (((p + 3) >> 2) + 3) & ~3;
      for (int a = p + lane; a < 4 * ks4; a += 64) sl[a] = 0.0;
      wave_lds_sync();
      // e2 = -(U_P^T s/(N-1) + epsbar), epsbar left in LDS by the Gram loop;
      // lane (q, c) sums members 16I + c over predecessors a = q mod 4, four
      // k-steps of loads at a time (pad row past p, columns 16I + c < ldu)
      const int nt = (N + 15) >> 4;
      double e[MT];
#pragma unroll
      for (int I = 0; I < MT; ++I) e[I] = 0.0;
      for (int ks0 = 0; ks0 < ks4; ks0 += 4) {
        double f[4][MT], sv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int a = 4 * (ks0 + u) + q;
          const int off = L.pidx[a] * ldu + c;
          sv[u] = sl[a];
#pragma unroll
          for (int I = 0; I < MT; ++I) f[u][I] = I < nt ? U[off + 16 * I] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int I = 0; I < MT; ++I) e[I] = fma(sv[u], f[u][I], e[I]);
      }
#pragma unroll
      for (int I = 0; I < MT; ++I) {
        if (I >= nt) break;
        double es = e[I];
        es = quarter_sum(es);
        const int k = 16 * I + c;
        if (q == 0 && k < N) adj.e2[r * N + k] = -(es / nm1 + adj.ebl[k]);
      }
    }
    ls = wave_sum(ls);
    if (lane == 0) adj.lam_row[r] = ls;
  }
}

// waves per SIMD each kernel is compiled for (register budget 512 / occupancy)
constexpr int occupancy_for(int T, bool KF) { return T <= 3 ? 4 : (T == 4 ? 3 : (T == 5 ? 2 : 1)); }

template <int T, bool KF, int MT>
__global__ __launch_bounds__(256, occupancy_for(T, KF)) void k_fit_batched(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, double lam, double *__restrict__ tval,
    double *__restrict__ dvec, int32_t *status, double *__restrict__ fcache, TileOut to) {
  __shared__ WaveLds<T> lds[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  WaveLds<T> &L = lds[wave];
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const int uoff = fit_glob[r] * ldu;
  if (!to.tiles) {
    for (int k = lane; k < kMaxP + 8; k += 64) L.pidx[k] = k < p ? fit_glob[B.row0 + col[lo + k]] : zrow;
  } else {
    // the predecessors' rows and each coefficient's place in the dense tiles,
    // from one read of the columns (the row tile's slots mapped first)
    const int local = (int)(r - B.row0);
    const int R = local >> 4, i = local & 15;
    const int64_t rt = B.rt0 + R;
    const int64_t t0 = to.rt_ptr[rt];
    const int nt = (int)(to.rt_ptr[rt + 1] - t0);
    for (int t = lane; t < nt; t += 64) {
      const int d = R - to.rt_col[t0 + t];
      if (d < kTileMapFit) L.tmap[d] = to.rt_slot[t0 + t];
    }
    wave_lds_sync();
    for (int k = lane; k < kMaxP + 8; k += 64) {
      if (k < p) {
        const int cc = col[lo + k];
        L.pidx[k] = fit_glob[B.row0 + cc];
        L.tdst[k] = tile_dest(to, R, i, rt, t0, nt, L.tmap, cc);
      } else {
        L.pidx[k] = zrow;
      }
    }
  }
  wave_lds_sync();
  if (!KF && lam == 0.0 && p >= N - 1) {
    if (lane == 0) set_error(status, ENKFMC_ENOTSPD, (int32_t)r);
    return;
  }
  double *fc = fcache ? fcache + (size_t)idx * (T * (T + 1) / 2) * 256 : nullptr;   // this row's cache slot
  fit_row<T, KF, MT>(lane, r, p, N, lam * (double)(N - 1), U, ldu, uoff, L, tval, lo, dvec, status, AdjIO{}, fc,
                     to.tiles, to.tdiag);
}

// Adjoint of the regressions of one bucket (same rows and shapes as the fit).
// The adjoint carries the pre- and post-pass values too: one wave per SIMD less
// for the larger kernel-form systems.
constexpr int adj_occupancy_for(int T, bool KF) {
  return KF ? (T <= 2 ? 4 : (T == 3 ? 3 : (T <= 5 ? 2 : 1))) : occupancy_for(T, KF);
}

template <int T, bool KF, int MT>
__global__ __launch_bounds__(256, adj_occupancy_for(T, KF)) void k_adj_regress_batched(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, double lam, double *__restrict__ tval,
    AdjIO adj, int32_t *status) {
  __shared__ WaveLds<T> lds[4];
  __shared__ double ebl[4][kMaxP + 8];   // epsbar (p-form, 16 kMaxT used) or b (kernel form)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  WaveLds<T> &L = lds[wave];
  const Block B = blocks[fit_blk[r]];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const int uoff = fit_glob[r] * ldu;
  for (int k = lane; k < kMaxP + 8; k += 64) L.pidx[k] = k < p ? fit_glob[B.row0 + col[lo + k]] : zrow;
  wave_lds_sync();
  AdjIO aw = adj;
  aw.ebl = ebl[wave];
  fit_row<T, KF, MT, true>(lane, r, p, N, lam * (double)(N - 1), U, ldu, uoff, L, tval, lo, nullptr, status, aw);
}

// waves per SIMD of the cached-factor solves (the tiles and the vector only)
constexpr int solve_occupancy_for(int T) { return T <= 3 ? 5 : (T == 4 ? 4 : (T == 5 ? 3 : 1)); }

// ---- kernel-form adjoint from the cached factor, in three launches ---------
// The recomputing adjoint (fit_row in ADJ mode) holds the Gram tiles in
// registers through its passes over U_P, at one or two wavefronts per SIMD,
// and those passes wait on their loads.  With the factor cached, the passes
// need no tiles and run as kernels of their own at high residency; only the
// solve holds the tiles, and it streams them from HBM once.
//   k_adj_kf_pre:   beta and b (push-through, as in adj_pre_kf), the sums
//                   eps = u - U_P^T beta and v = U_P^T b; writes e1, epsbar
//                   (into e2) and v (into vbuf);
//   k_adj_kf_solve: the row's tiles from the cache, y = L^-1 v, x = L^-T y
//                   (x overwrites v in vbuf);
//   k_adj_kf_post:  s = (N-1)/mu (b - U_P x) (into sb), the row's share of
//                   dL/dlam, g = U_P^T s, e2 = -(g/(N-1) + epsbar).
// vbuf holds N doubles per fit row (row r at r N).

// Predecessor rows of fit row r into pidx (the pad row past p).
__device__ __forceinline__ void load_pidx(const int lane, const int64_t r, const Block *__restrict__ blocks,
                                          const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
                                          const int32_t *__restrict__ col, const int64_t lo, const int p,
                                          const int zrow, int *pidx) {
  const Block B = blocks[fit_blk[r]];
  for (int k = lane; k < kMaxP + 8; k += 64) pidx[k] = k < p ? fit_glob[B.row0 + col[lo + k]] : zrow;
  wave_lds_sync();
}

template <int T>
__global__ __launch_bounds__(256) void k_adj_kf_pre(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, double lam, const double *__restrict__ tval,
    AdjIO adj, double *__restrict__ vbuf) {
  __shared__ int spidx[4][kMaxP + 8];
  __shared__ double sbeta[4][kMaxP + 8], sb[4][kMaxP + 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const int uoff = fit_glob[r] * ldu;
  int *pidx = spidx[wave];
  double *bl = sbeta[wave], *bv = sb[wave];
  const double nm1 = (double)(N - 1), mu = lam * nm1, Db = adj.dbar[r];
  const double coef = 2.0 * Db * mu / nm1;
  for (int a = lane; a < kMaxP + 8; a += 64) {
    const double beta = a < p ? -tval[lo + a] : 0.0;
    const double b = a < p ? fma(-coef, beta, adj.sb[lo + a]) : 0.0;
    bl[a] = beta;
    bv[a] = b;
    if (a < p) adj.sb[lo + a] = b;
  }
  load_pidx(lane, r, blocks, fit_glob, fit_blk, col, lo, p, zrow, pidx);
  // lane (q, c) sums beta_a U[P_a][k] and b_a U[P_a][k] over predecessors
  // a = 4ks + q for members k = 16I + c, four k-steps of loads per trip
  // (past p: the zero pad row, beta = b = 0; 4 * 48 <= kMaxP)
  double ea[T], ta[T];
#pragma unroll
  for (int I = 0; I < T; ++I) ea[I] = ta[I] = 0.0;
  const int ks4 = (((p + 3) >> 2) + 3) & ~3;
  for (int ks0 = 0; ks0 < ks4; ks0 += 4) {
    double f[4][T];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int off = pidx[4 * (ks0 + u) + q] * ldu + c;
#pragma unroll
      for (int I = 0; I < T; ++I) f[u][I] = U[off + 16 * I];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double bb = bl[4 * (ks0 + u) + q], bw = bv[4 * (ks0 + u) + q];
#pragma unroll
      for (int I = 0; I < T; ++I) {
        ea[I] = fma(bb, f[u][I], ea[I]);
        ta[I] = fma(bw, f[u][I], ta[I]);
      }
    }
  }
#pragma unroll
  for (int I = 0; I < T; ++I) {
    const double es = quarter_sum(ea[I]);
    const double tb = quarter_sum(ta[I]);
    const int k = 16 * I + c;
    if (q == 0 && k < N) {
      const double eps = U[uoff + k] - es;
      adj.e1[r * N + k] = eps / nm1;
      adj.e2[r * N + k] = 2.0 * Db * eps / nm1;
      vbuf[r * N + k] = tb;
    }
  }
}

template <int T>
__global__ __launch_bounds__(256, solve_occupancy_for(T)) void k_adj_kf_solve(
    const int32_t *__restrict__ rows, int64_t nrows, int N, const double *__restrict__ fcache,
    double *__restrict__ vbuf) {
  constexpr int NT = T * (T + 1) / 2;
  __shared__ double svec[4][16 * (T + 1)];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const double *fc = fcache + (size_t)idx * NT * 256;   // the fit's slot of this row
  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double2 *src = (const double2 *)(fc + (size_t)(64 * t + lane) * 4);
    const double2 a01 = src[0], a23 = src[1];
    acc[t] = d4{a01.x, a01.y, a23.x, a23.y};
  }
  double vr[T];
#pragma unroll
  for (int J = 0; J < T; ++J) vr[J] = (q == 0 && 16 * J + c < N) ? vbuf[r * N + 16 * J + c] : 0.0;
  double *y = svec[wave];
  fwd_subst<T>(q, c, acc, vr, y, y + 16 * T);
  back_subst<T>(q, c, acc, vr, y);
  for (int k = lane; k < N; k += 64) vbuf[r * N + k] = y[k];
}

template <int T>
__global__ __launch_bounds__(256) void k_adj_kf_post(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, double lam, const double *__restrict__ tval,
    AdjIO adj, const double *__restrict__ vbuf) {
  __shared__ int spidx[4][kMaxP + 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  int *pidx = spidx[wave];
  load_pidx(lane, r, blocks, fit_glob, fit_blk, col, lo, p, zrow, pidx);
  const double nm1 = (double)(N - 1), mu = lam * nm1;
  // s_a = (N-1)/mu (b_a - sum_k U[P_a][k] x_k) and g = U_P^T s from the same
  // fragments: lane (q, c) loads members 16I + c of predecessor 4ks + q, and
  // the 16 lanes of each quarter add their partial sums
  double wv[T], gacc[T];
#pragma unroll
  for (int I = 0; I < T; ++I) {
    wv[I] = 16 * I + c < N ? vbuf[r * N + 16 * I + c] : 0.0;
    gacc[I] = 0.0;
  }
  double ls = 0.0;
  const int ks4 = (((p + 3) >> 2) + 3) & ~3;
  for (int ks0 = 0; ks0 < ks4; ks0 += 4) {
    double f[4][T], sbv[4], tv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = 4 * (ks0 + u) + q;
      const int off = pidx[a] * ldu + c;
#pragma unroll
      for (int I = 0; I < T; ++I) f[u][I] = U[off + 16 * I];
      sbv[u] = a < p ? adj.sb[lo + a] : 0.0;
      tv[u] = a < p ? tval[lo + a] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = 4 * (ks0 + u) + q;
      double b = 0.0;
#pragma unroll
      for (int I = 0; I < T; ++I) b = fma(f[u][I], wv[I], b);
      b = row16_sum(b);
      const double sv = a < p ? (nm1 / mu) * (sbv[u] - b) : 0.0;
      if (c == 0 && a < p) {
        adj.sb[lo + a] = sv;
        ls = fma(sv, tv[u], ls);
      }
#pragma unroll
      for (int I = 0; I < T; ++I) gacc[I] = fma(f[u][I], sv, gacc[I]);
    }
  }
#pragma unroll
  for (int I = 0; I < T; ++I) {
    const double e = quarter_sum(gacc[I]);
    const int k = 16 * I + c;
    if (q == 0 && k < N) adj.e2[r * N + k] = -(e / nm1 + adj.e2[r * N + k]);
  }
  ls = wave_sum(ls);
  if (lane == 0) adj.lam_row[r] = ls;
}

// ---- p-form adjoint from the cached factor, in three launches ------------
//   k_adj_pf_pre:   eps_k = u_k - sum_a beta_a U[P_a][k], e1, epsbar (into
//                   e2) and b = betabar - U_P epsbar (into vbuf), one pass
//                   over the members;
//   k_adj_pf_solve: the row's tiles from the cache, x = G^-1 b by forward and
//                   back substitution, s = (N-1) x (into sb) and the row's
//                   share of dL/dlam;
//   k_adj_pf_post:  e2 = -(U_P^T s/(N-1) + epsbar), one pass over the
//                   predecessors.
template <int T>
__global__ __launch_bounds__(256) void k_adj_pf_pre(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, const double *__restrict__ tval, AdjIO adj,
    double *__restrict__ vbuf) {
  __shared__ int spidx[4][kMaxP + 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const int uoff = fit_glob[r] * ldu;
  int *pidx = spidx[wave];
  load_pidx(lane, r, blocks, fit_glob, fit_blk, col, lo, p, zrow, pidx);
  const double nm1 = (double)(N - 1), Db = adj.dbar[r];
  // lane (q, c) holds beta of predecessor 16I + c; one 16-byte load per tile
  // brings members 8ks + 2q and 8ks + 2q + 1 (8 * ks2 <= ldu); the 16 lanes
  // of a quarter sum beta_a U[P_a][k] for its two members, and vp[I] gathers
  // sum_k U[P_{16I+c}][k] epsbar_k
  int base[T];
  double bet[T], vp[T];
#pragma unroll
  for (int I = 0; I < T; ++I) {
    base[I] = pidx[16 * I + c] * ldu + 2 * q;
    bet[I] = 16 * I + c < p ? -tval[lo + 16 * I + c] : 0.0;
    vp[I] = 0.0;
  }
  const int ks2 = (N + 7) >> 3;
  for (int ks = 0; ks < ks2; ++ks) {
    double2 f[T];
#pragma unroll
    for (int I = 0; I < T; ++I) f[I] = *(const double2 *)&U[base[I] + 8 * ks];
    const double2 uk = *(const double2 *)&U[uoff + 2 * q + 8 * ks];
    double es0 = 0.0, es1 = 0.0;
#pragma unroll
    for (int I = 0; I < T; ++I) {
      es0 = fma(bet[I], f[I].x, es0);
      es1 = fma(bet[I], f[I].y, es1);
    }
    es0 = row16_sum(es0);
    es1 = row16_sum(es1);
    const int k0 = 8 * ks + 2 * q, k1 = k0 + 1;
    const double eps0 = k0 < N ? uk.x - es0 : 0.0, eps1 = k1 < N ? uk.y - es1 : 0.0;
    const double eb0 = 2.0 * Db * eps0 / nm1, eb1 = 2.0 * Db * eps1 / nm1;
    if (c == 0 && k0 < N) {
      adj.e1[r * N + k0] = eps0 / nm1;
      adj.e2[r * N + k0] = eb0;
    }
    if (c == 0 && k1 < N) {
      adj.e1[r * N + k1] = eps1 / nm1;
      adj.e2[r * N + k1] = eb1;
    }
#pragma unroll
    for (int I = 0; I < T; ++I) vp[I] = fma(f[I].y, eb1, fma(f[I].x, eb0, vp[I]));
  }
#pragma unroll
  for (int I = 0; I < T; ++I) {
    const double v = quarter_sum(vp[I]);
    const int a = 16 * I + c;
    if (q == 0 && a < p) vbuf[r * N + a] = adj.sb[lo + a] - v;   // b_a
  }
}

template <int T>
__global__ __launch_bounds__(256, solve_occupancy_for(T)) void k_adj_pf_solve(
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ rows, int64_t nrows, int N,
    const double *__restrict__ tval, const double *__restrict__ fcache, const double *__restrict__ vbuf, AdjIO adj) {
  constexpr int NT = T * (T + 1) / 2;
  __shared__ double svec[4][16 * (T + 1)];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  const double *fc = fcache + (size_t)idx * NT * 256;   // the fit's slot of this row
  d4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double2 *src = (const double2 *)(fc + (size_t)(64 * t + lane) * 4);
    const double2 a01 = src[0], a23 = src[1];
    acc[t] = d4{a01.x, a01.y, a23.x, a23.y};
  }
  double vr[T];
#pragma unroll
  for (int J = 0; J < T; ++J) vr[J] = (q == 0 && 16 * J + c < p) ? vbuf[r * N + 16 * J + c] : 0.0;
  double *y = svec[wave];
  fwd_subst<T>(q, c, acc, vr, y, y + 16 * T);
  back_subst<T>(q, c, acc, vr, y);
  // s = (N-1) x overwrites betabar in sb (now b, read by the pre-pass)
  const double nm1 = (double)(N - 1);
  double ls = 0.0;
  for (int a = lane; a < p; a += 64) {
    const double sv = nm1 * y[a];
    adj.sb[lo + a] = sv;
    ls = fma(sv, tval[lo + a], ls);
  }
  ls = wave_sum(ls);
  if (lane == 0) adj.lam_row[r] = ls;
}

template <int T, int MT>
__global__ __launch_bounds__(256) void k_adj_pf_post(
    const Block *__restrict__ blocks, const int32_t *__restrict__ fit_glob, const int32_t *__restrict__ fit_blk,
    const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ U, int ldu,
    int N, const int32_t *__restrict__ rows, int64_t nrows, int zrow, AdjIO adj) {
  __shared__ int spidx[4][kMaxP + 8];
  __shared__ double ssl[4][kMaxP + 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const int64_t lo = row_ptr[r];
  const int p = (int)(row_ptr[r + 1] - lo);
  int *pidx = spidx[wave];
  double *sl = ssl[wave];   // s, zero past p
  for (int a = lane; a < kMaxP + 8; a += 64) sl[a] = a < p ? adj.sb[lo + a] : 0.0;
  load_pidx(lane, r, blocks, fit_glob, fit_blk, col, lo, p, zrow, pidx);
  // lane (q, c) sums members 16I + c over predecessors a = q mod 4, four
  // k-steps of loads at a time (pad row past p, columns 16I + c < ldu)
  const double nm1 = (double)(N - 1);
  const int nt = (N + 15) >> 4;
  const int ks4 = (((p + 3) >> 2) + 3) & ~3;
  double e[MT];
#pragma unroll
  for (int I = 0; I < MT; ++I) e[I] = 0.0;
  for (int ks0 = 0; ks0 < ks4; ks0 += 4) {
    double f[4][MT], sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = 4 * (ks0 + u) + q;
      const int off = pidx[a] * ldu + c;
      sv[u] = sl[a];
#pragma unroll
      for (int I = 0; I < MT; ++I) f[u][I] = I < nt ? U[off + 16 * I] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int I = 0; I < MT; ++I) e[I] = fma(sv[u], f[u][I], e[I]);
  }
#pragma unroll
  for (int I = 0; I < MT; ++I) {
    if (I >= nt) break;
    const double es = quarter_sum(e[I]);
    const int k = 16 * I + c;
    if (q == 0 && k < N) adj.e2[r * N + k] = -(es / nm1 + adj.e2[r * N + k]);
  }
}

// Adjoint of the regressions without predecessors (eps = u).
__global__ __launch_bounds__(256) void k_adj_p0(const int32_t *__restrict__ fit_glob, const double *__restrict__ U,
                                                int ldu, int N, const int32_t *__restrict__ rows, int64_t nrows,
                                                AdjIO adj) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const double *u = U + (int64_t)fit_glob[r] * ldu;
  const double nm1 = (double)(N - 1), Db = adj.dbar[r];
  for (int cc = lane; cc < N; cc += 64) {
    adj.e1[r * N + cc] = u[cc] / nm1;
    adj.e2[r * N + cc] = -2.0 * Db * u[cc] / nm1;
  }
  if (lane == 0) adj.lam_row[r] = 0.0;
}

// Regressions without predecessors: d = u^T u / (N - 1).
__global__ __launch_bounds__(256) void k_fit_p0(const int32_t *__restrict__ fit_glob, const double *__restrict__ U,
                                                int ldu, int N, const int32_t *__restrict__ rows, int64_t nrows,
                                                double *__restrict__ dvec, int32_t *status) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t idx = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wave;
  if (idx >= nrows) return;
  const int64_t r = rows[idx];
  const double *u = U + (int64_t)fit_glob[r] * ldu;
  double s = 0.0;
  for (int cc = lane; cc < N; cc += 64) s += u[cc] * u[cc];
  s = wave_sum(s);
  if (lane == 0) {
    const double dd = s / (N - 1);
    dvec[r] = dd;
    if (!(dd > 0.0)) set_error(status, ENKFMC_ENONPOS_D, (int32_t)r);
  }
}

// The tiles of T are written by the fit when every row runs a one-wavefront
// kernel (no plain bucket); otherwise k_build_tiles assembles them after it.
// (destinations are 32-bit indices: at most 2^31 / 256 tiles)
bool fit_writes_tiles(const enkfmc_plan *p) {
  return p->bucket_off[kBucketPlain + 1] == p->bucket_off[kBucketPlain] && (int64_t)p->n_slots < (1ll << 23) &&
         (int64_t)p->n_rt < (1ll << 23);
}

// Cholesky factor of one block's S = R + F^T D F (up to 128 observations) by
// chol_tiles, one wavefront per block.  The lower triangle of S loads into
// the registers as chol_tiles expects them (tile (I, J) transposed; the
// diagonal tiles from their lower halves, mirrored), entries at or past row
// or column m as the identity; the factor goes back to S in its natural
// layout: L_IJ from the factored tiles, L_JJ as the diagonal tiles leave the
// elimination.
template <int T>
__device__ __forceinline__ bool dual_chol_block(const int q, const int c, const Block &B, double *__restrict__ S) {
  constexpr int NT = T * (T + 1) / 2;
  const int m = B.m;
  const int64_t ldf = B.ldf;
  double *L = S + B.S0;
  d4 acc[NT];
#pragma unroll
  for (int I = 0; I < T; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int i = 16 * I + c, j = 16 * J + 4 * rr + q;   // element (4rr + q, c) of A_IJ^T is A[i][j]
        const int hi = i > j ? i : j, lo = i > j ? j : i;
        const double v = L[hi * ldf + lo];
        acc[tix<T>(I, J)][rr] = (hi < m) ? v : (i == j ? 1.0 : 0.0);
      }
  double augv[T];
#pragma unroll
  for (int J = 0; J < T; ++J) augv[J] = 0.0;
  const auto diag_out = [&](int J, const d4 &t) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
      if (4 * rr + q >= c) L[(16 * J + 4 * rr + q) * ldf + 16 * J + c] = t[rr];
  };
  if (!chol_tiles<T, false>(q, c, m, acc, augv, nullptr, diag_out)) return false;
#pragma unroll
  for (int I = 1; I < T; ++I)
#pragma unroll
    for (int J = 0; J < I; ++J)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) L[(16 * I + c) * ldf + 16 * J + 4 * rr + q] = acc[tix<T>(I, J)][rr];
  return true;
}

__global__ __launch_bounds__(64, 1) void k_dual_chol_tiles(const Block *__restrict__ blocks, double *__restrict__ S,
                                                          int32_t *status) {
  const Block B = blocks[blockIdx.x];
  if (B.m == 0) return;
  const int lane = threadIdx.x, q = lane >> 4, c = lane & 15;
  bool ok;
  switch ((B.m + 15) >> 4) {
    case 1: ok = dual_chol_block<1>(q, c, B, S); break;
    case 2: ok = dual_chol_block<2>(q, c, B, S); break;
    case 3: ok = dual_chol_block<3>(q, c, B, S); break;
    case 4: ok = dual_chol_block<4>(q, c, B, S); break;
    case 5: ok = dual_chol_block<5>(q, c, B, S); break;
    case 6: ok = dual_chol_block<6>(q, c, B, S); break;
    case 7: ok = dual_chol_block<7>(q, c, B, S); break;
    default: ok = dual_chol_block<8>(q, c, B, S); break;
  }
  if (!ok && lane == 0) set_error(status, ENKFMC_ENOTSPD, -1 - (int32_t)blockIdx.x);
}

bool dual_chol_tiles_fit(const enkfmc_plan *p) { return p->max_bm <= 16 * kMaxT; }

hipError_t launch_dual_chol_tiles(enkfmc_plan *p, const Dev &d, hipStream_t s) {
  hipLaunchKernelGGL(k_dual_chol_tiles, dim3((unsigned)p->blocks.size()), dim3(64), 0, s, d.blocks, d.S, d.status);
  return hipGetLastError();
}

static TileOut tile_out(const enkfmc_plan *p, const Dev &d) {
  return TileOut{fit_writes_tiles(p) ? d.tiles : nullptr, d.tdiag, d.rt_ptr, d.rt_col, d.rt_slot, d.col};
}

template <int T, bool KF, int MT>
static void launch_bucket(enkfmc_plan *p, const Dev &d, const int32_t *rows, int64_t n, double lam, hipStream_t s,
                          double *fcache = nullptr) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fit_batched<T, KF, MT>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, d.blocks,
                     d.fit_glob, d.fit_blk, d.row_ptr, d.col, d.U, p->ldu, p->N, rows, n, (int)p->n, lam, d.tval,
                     d.dvec, d.status, fcache, tile_out(p, d));
}

// p-form bucket of T tiles: the residual loops unroll 5 member tiles when
// N <= 80, else 8.
template <int T>
static void launch_pform(enkfmc_plan *p, const Dev &d, const int32_t *rows, int64_t n, double lam, hipStream_t s) {
  double *fc = p->fcache ? p->fcache + fcache_offset(p, T) : nullptr;   // NULL: no factor cache
  if constexpr (T <= 5) {
    if (p->N <= 80) return launch_bucket<T, false, 5>(p, d, rows, n, lam, s, fc);
  }
  launch_bucket<T, false, 8>(p, d, rows, n, lam, s, fc);
}

hipError_t launch_fit_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  phase_begin(p, ENKFMC_PH_FIT, s);
  const int32_t *rows = d.fit_rows;
  const int64_t *bo = p->bucket_off;   // see kBucket* in plan.h
  if (bo[kBucketP0 + 1] > bo[kBucketP0])
    hipLaunchKernelGGL(k_fit_p0, dim3((unsigned)((bo[kBucketP0 + 1] - bo[kBucketP0] + 3) / 4)), dim3(256), 0, s,
                       d.fit_glob, d.U, p->ldu, p->N, rows + bo[kBucketP0], bo[kBucketP0 + 1] - bo[kBucketP0], d.dvec,
                       d.status);
  auto nb = [&](int b) { return bo[b + 1] - bo[b]; };
  launch_pform<1>(p, d, rows + bo[1], nb(1), lam, s);
  launch_pform<2>(p, d, rows + bo[2], nb(2), lam, s);
  launch_pform<3>(p, d, rows + bo[3], nb(3), lam, s);
  launch_pform<4>(p, d, rows + bo[4], nb(4), lam, s);
  launch_pform<5>(p, d, rows + bo[5], nb(5), lam, s);
  launch_pform<6>(p, d, rows + bo[6], nb(6), lam, s);
  launch_pform<7>(p, d, rows + bo[7], nb(7), lam, s);
  launch_pform<8>(p, d, rows + bo[8], nb(8), lam, s);
  const int64_t nk = nb(kBucketKF);
  const int32_t *rk = rows + bo[kBucketKF];
  if (nk > 0) {
    // kernel form: m = N.  Without a ridge these rows (p >= N) are ENOTSPD,
    // which the p-form kernel reports before any arithmetic.
    if (lam > 0.0) {
      double *fc = p->fcache ? p->fcache + fcache_offset(p, kBucketKF) : nullptr;   // NULL: no factor cache
      phase_begin(p, ENKFMC_PH_FIT_KFORM, s);
      switch ((p->N + 15) / 16) {
        case 1: launch_bucket<1, true, 1>(p, d, rk, nk, lam, s, fc); break;
        case 2: launch_bucket<2, true, 2>(p, d, rk, nk, lam, s, fc); break;
        case 3: launch_bucket<3, true, 3>(p, d, rk, nk, lam, s, fc); break;
        case 4: launch_bucket<4, true, 4>(p, d, rk, nk, lam, s, fc); break;
        case 5: launch_bucket<5, true, 5>(p, d, rk, nk, lam, s, fc); break;
        case 6: launch_bucket<6, true, 6>(p, d, rk, nk, lam, s, fc); break;
        case 7: launch_bucket<7, true, 7>(p, d, rk, nk, lam, s, fc); break;
        default: launch_bucket<8, true, 8>(p, d, rk, nk, lam, s, fc); break;
      }
      phase_end(p, ENKFMC_PH_FIT_KFORM, s);
    } else {
      launch_bucket<1, false, 8>(p, d, rk, nk, lam, s);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // rows no one-wavefront kernel takes: the plain kernel, on those rows only
  if (nb(kBucketPlain) > 0) {
    phase_begin(p, ENKFMC_PH_FIT_FALLBACK, s);
    e = launch_fit_plain_rows(p, d, lam, d.fit_rows + bo[kBucketPlain], nb(kBucketPlain), s);
    phase_end(p, ENKFMC_PH_FIT_FALLBACK, s);
    if (e != hipSuccess) return e;
  }
  phase_end(p, ENKFMC_PH_FIT, s);
  return hipGetLastError();
}

template <int T, bool KF, int MT>
static void launch_adj_bucket(enkfmc_plan *p, const Dev &d, const int32_t *rows, int64_t n, double lam,
                              const AdjIO &adj, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_adj_regress_batched<T, KF, MT>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, d.blocks,
                     d.fit_glob, d.fit_blk, d.row_ptr, d.col, d.U, p->ldu, p->N, rows, n, (int)p->n, lam, d.tval,
                     adj, d.status);
}

// Kernel-form adjoint of T tiles, from the fit's cached factors when it left them.
template <int T>
static void launch_adj_kform(enkfmc_plan *p, const Dev &d, const int32_t *rows, int64_t n, double lam,
                             const AdjIO &adj, hipStream_t s) {
  if (n <= 0) return;
  if (!p->fcache_valid) return launch_adj_bucket<T, true, T>(p, d, rows, n, lam, adj, s);
  // the cached factor: two passes over U_P and the solve between them, with
  // v and then x in the Ubar buffer (not in use until the gather)
  const dim3 g((unsigned)((n + 3) / 4));
  hipLaunchKernelGGL(k_adj_kf_pre<T>, g, dim3(256), 0, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr, d.col, d.U,
                     p->ldu, p->N, rows, n, (int)p->n, lam, d.tval, adj, d.ubar);
  hipLaunchKernelGGL(k_adj_kf_solve<T>, g, dim3(256), 0, s, rows, n, p->N,
                     (const double *)p->fcache + fcache_offset(p, kBucketKF), d.ubar);
  hipLaunchKernelGGL(k_adj_kf_post<T>, g, dim3(256), 0, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr, d.col, d.U,
                     p->ldu, p->N, rows, n, (int)p->n, lam, d.tval, adj, (const double *)d.ubar);
}

template <int T>
static void launch_adj_pform(enkfmc_plan *p, const Dev &d, const int32_t *rows, int64_t n, double lam,
                             const AdjIO &adj, hipStream_t s) {
  if (n <= 0) return;
  if (p->fcache_valid) {
    // the cached factor: pass over U_P^T, solve, pass over U_P (v, then s,
    // in the Ubar buffer and in sb)
    const dim3 g((unsigned)((n + 3) / 4));
    hipLaunchKernelGGL(k_adj_pf_pre<T>, g, dim3(256), 0, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr, d.col, d.U,
                       p->ldu, p->N, rows, n, (int)p->n, (const double *)d.tval, adj, d.ubar);
    hipLaunchKernelGGL(k_adj_pf_solve<T>, g, dim3(256), 0, s, d.row_ptr, rows, n, p->N, (const double *)d.tval,
                       (const double *)p->fcache + fcache_offset(p, T), (const double *)d.ubar, adj);
    if (T <= 5 && p->N <= 80)
      hipLaunchKernelGGL((k_adj_pf_post<T, 5>), g, dim3(256), 0, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr, d.col,
                         d.U, p->ldu, p->N, rows, n, (int)p->n, adj);
    else
      hipLaunchKernelGGL((k_adj_pf_post<T, 8>), g, dim3(256), 0, s, d.blocks, d.fit_glob, d.fit_blk, d.row_ptr, d.col,
                         d.U, p->ldu, p->N, rows, n, (int)p->n, adj);
    return;
  }
  if constexpr (T <= 5) {
    if (p->N <= 80) return launch_adj_bucket<T, false, 5>(p, d, rows, n, lam, adj, s);
  }
  launch_adj_bucket<T, false, 8>(p, d, rows, n, lam, adj, s);
}

// Adjoint of every regression over the fit's buckets; the rows of the plain
// bucket go to the plain per-row adjoint.
hipError_t launch_adj_regress_batched(enkfmc_plan *p, const Dev &d, double lam, hipStream_t s) {
  const AdjIO adj{d.dbar, d.aux3, d.aux1, d.aux2, d.red};
  const int32_t *rows = d.fit_rows;
  const int64_t *bo = p->bucket_off;
  auto nb = [&](int b) { return bo[b + 1] - bo[b]; };
  if (nb(kBucketP0) > 0)
    hipLaunchKernelGGL(k_adj_p0, dim3((unsigned)((nb(kBucketP0) + 3) / 4)), dim3(256), 0, s, d.fit_glob, d.U,
                       p->ldu, p->N, rows + bo[kBucketP0], nb(kBucketP0), adj);
  launch_adj_pform<1>(p, d, rows + bo[1], nb(1), lam, adj, s);
  launch_adj_pform<2>(p, d, rows + bo[2], nb(2), lam, adj, s);
  launch_adj_pform<3>(p, d, rows + bo[3], nb(3), lam, adj, s);
  launch_adj_pform<4>(p, d, rows + bo[4], nb(4), lam, adj, s);
  launch_adj_pform<5>(p, d, rows + bo[5], nb(5), lam, adj, s);
  launch_adj_pform<6>(p, d, rows + bo[6], nb(6), lam, adj, s);
  launch_adj_pform<7>(p, d, rows + bo[7], nb(7), lam, adj, s);
  launch_adj_pform<8>(p, d, rows + bo[8], nb(8), lam, adj, s);
  const int64_t nk = nb(kBucketKF);
  const int32_t *rk = rows + bo[kBucketKF];
  if (nk > 0) {
    if (!(lam > 0.0)) return hipErrorInvalidValue;   // the fit rejects p >= N - 1 without ridge
    switch ((p->N + 15) / 16) {
      case 1: launch_adj_kform<1>(p, d, rk, nk, lam, adj, s); break;
      case 2: launch_adj_kform<2>(p, d, rk, nk, lam, adj, s); break;
      case 3: launch_adj_kform<3>(p, d, rk, nk, lam, adj, s); break;
      case 4: launch_adj_kform<4>(p, d, rk, nk, lam, adj, s); break;
      case 5: launch_adj_kform<5>(p, d, rk, nk, lam, adj, s); break;
      case 6: launch_adj_kform<6>(p, d, rk, nk, lam, adj, s); break;
      case 7: launch_adj_kform<7>(p, d, rk, nk, lam, adj, s); break;
      default: launch_adj_kform<8>(p, d, rk, nk, lam, adj, s); break;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb(kBucketPlain) > 0) return launch_adj_regress_plain_rows(p, d, lam, rows + bo[kBucketPlain],
                                                                 nb(kBucketPlain), s);
  return hipSuccess;
}

}  // namespace enkfmc
