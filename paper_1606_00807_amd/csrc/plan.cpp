// Host planner: sub-domain decomposition, local ordering, radius-restricted
// predecessor pattern and local observation lists (Section 3 and the text
// after eq. 9 of arXiv 1606.00807; Alg. 2 decomposition step).  Integer
// arithmetic only; runs once per geometry.
#include <algorithm>
#include <cstdlib>

#include "plan.h"

namespace enkfmc {

static void tile_bounds(int32_t extent, int32_t tiles, int32_t k, int32_t *s, int32_t *e) {
  int32_t base = extent / tiles, rem = extent % tiles;
  *s = k * base + std::min(k, rem);
  *e = *s + base + (k < rem ? 1 : 0);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

enkfmc_status build_plan(enkfmc_plan *p, const enkfmc_geometry *g, int32_t N, const int32_t *obs_idx, int32_t m,
                         std::string *err) {
  if (!g || !g->nlev) { *err = "geometry or nlev is NULL"; return ENKFMC_EINVAL; }
  if (g->nx < 1 || g->ny < 1 || g->nvar < 1 || g->sdx < 1 || g->sdy < 1 || g->sdx > g->nx || g->sdy > g->ny) {
    *err = "grid, variable or tile counts out of range"; return ENKFMC_EINVAL;
  }
  if (g->r_h < 0 || g->r_v < 0) { *err = "negative radius"; return ENKFMC_EINVAL; }
  if (N < 2) { *err = "ensemble size N must be >= 2"; return ENKFMC_EINVAL; }
  if (m < 0 || (m > 0 && !obs_idx)) { *err = "bad observation list"; return ENKFMC_EINVAL; }
  p->nx = g->nx; p->ny = g->ny; p->nvar = g->nvar; p->periodic_x = g->periodic_x ? 1 : 0;
  p->sdx = g->sdx; p->sdy = g->sdy; p->r_h = g->r_h; p->r_v = g->r_v; p->N = N;
  p->ldu = (N + 15) / 16 * 16;
  p->nlev.assign(g->nlev, g->nlev + g->nvar);
  p->var_off.resize(g->nvar);
  int64_t n = 0;
  for (int v = 0; v < g->nvar; ++v) {
    if (p->nlev[v] < 1) { *err = "every variable needs >= 1 level"; return ENKFMC_EINVAL; }
    p->var_off[v] = (int32_t)n;
    n += (int64_t)g->nx * g->ny * p->nlev[v];
  }
  if (n >= (int64_t(1) << 31)) { *err = "state too large for 32-bit component indices"; return ENKFMC_EUNSUPPORTED; }
  p->n = n;
  p->m = m;
  p->obs_idx.assign(obs_idx ? obs_idx : nullptr, obs_idx ? obs_idx + m : nullptr);
  for (int32_t o = 0; o < m; ++o) {
    if (obs_idx[o] < 0 || obs_idx[o] >= n || (o > 0 && obs_idx[o] <= obs_idx[o - 1])) {
      *err = "obs_idx must be strictly increasing inside [0, n)"; return ENKFMC_EINVAL;
    }
  }
  const bool ring = p->periodic_x && p->sdx == 1;
  if (p->periodic_x && p->sdx > 1) {
    int32_t s, e;
    tile_bounds(p->nx, p->sdx, 0, &s, &e);
    if ((e - s) + 2 * p->r_h > p->nx) { *err = "longitude halo wraps onto its own tile"; return ENKFMC_EINVAL; }
  }
  const int32_t nsd = p->sdx * p->sdy;
  p->subs.clear(); p->blocks.clear();
  p->fit_glob.clear(); p->fit_blk.clear(); p->col.clear();
  p->row_ptr.assign(1, 0);
  p->interior_src.assign(n, -1);
  int64_t n_fit = 0;
  for (int32_t k = 0; k < nsd; ++k) {
    SubBox sb{};
    sb.kx = k % p->sdx; sb.ky = k / p->sdx;
    tile_bounds(p->nx, p->sdx, sb.kx, &sb.x0, &sb.x1);
    tile_bounds(p->ny, p->sdy, sb.ky, &sb.y0, &sb.y1);
    sb.ring = ring;
    if (ring) { sb.xs = 0; sb.BX = p->nx; }
    else if (p->periodic_x) { sb.xs = sb.x0 - p->r_h; sb.BX = (sb.x1 - sb.x0) + 2 * p->r_h; }
    else { sb.xs = std::max(0, sb.x0 - p->r_h); sb.BX = std::min(p->nx, sb.x1 + p->r_h) - sb.xs; }
    sb.ys = std::max(0, sb.y0 - p->r_h);
    sb.BY = std::min(p->ny, sb.y1 + p->r_h) - sb.ys;
    sb.blk0 = (int32_t)p->blocks.size();
    int32_t sd_row = 0;
    int64_t nz_sd0 = (int64_t)p->col.size();
    for (int32_t v = 0; v < p->nvar; ++v) {
      Block b{};
      b.sd = k; b.var = v; b.nlev = p->nlev[v]; b.BY = sb.BY; b.BX = sb.BX;
      b.n = b.nlev * b.BY * b.BX; b.sd_row0 = sd_row; b.row0 = n_fit; b.nz0 = (int64_t)p->col.size();
      const int32_t bid = (int32_t)p->blocks.size();
      for (int32_t l = 0; l < b.nlev; ++l)
        for (int32_t iy = 0; iy < b.BY; ++iy)
          for (int32_t ix = 0; ix < b.BX; ++ix) {
            const int32_t r = (l * b.BY + iy) * b.BX + ix;
            const int32_t glat = sb.ys + iy;
            const int32_t glon = ((sb.xs + ix) % p->nx + p->nx) % p->nx;
            const int32_t gidx = p->var_off[v] + (l * p->ny + glat) * p->nx + glon;
            p->fit_glob.push_back(gidx);
            p->fit_blk.push_back(bid);
            const bool in_lon = ring || (sb.x0 <= sb.xs + ix && sb.xs + ix < sb.x1);
            if (in_lon && sb.y0 <= glat && glat < sb.y1) {
              if (p->interior_src[gidx] != -1) { *err = "internal: component mapped back twice"; return ENKFMC_EINVAL; }
              p->interior_src[gidx] = (int32_t)(b.row0 + r);
            }
            // predecessors: same variable, inside the local box, earlier in local order
            const int32_t l_lo = std::max(0, l - p->r_v), l_hi = std::min(b.nlev - 1, l + p->r_v);
            const int32_t y_lo = std::max(0, iy - p->r_h), y_hi = std::min(b.BY - 1, iy + p->r_h);
            const int32_t x_lo = ring ? 0 : std::max(0, ix - p->r_h);
            const int32_t x_hi = ring ? b.BX - 1 : std::min(b.BX - 1, ix + p->r_h);
            int32_t cnt = 0;
            for (int32_t l2 = l_lo; l2 <= l_hi; ++l2)
              for (int32_t y2 = y_lo; y2 <= y_hi; ++y2)
                for (int32_t x2 = x_lo; x2 <= x_hi; ++x2) {
                  if (ring) {
                    int32_t dd = std::abs(ix - x2);
                    dd = std::min(dd, p->nx - dd);
                    if (dd > p->r_h) continue;
                  }
                  const int32_t r2 = (l2 * b.BY + y2) * b.BX + x2;
                  if (r2 < r) { p->col.push_back(r2); ++cnt; }
                }
            p->max_p = std::max(p->max_p, cnt);
            p->row_ptr.push_back((int64_t)p->col.size());
          }
      n_fit += b.n;
      sd_row += b.n;
      p->max_bn = std::max(p->max_bn, b.n);
      p->blocks.push_back(b);
    }
    sb.n_sd = sd_row;
    sb.nnz_sd = (int64_t)p->col.size() - nz_sd0;
    p->subs.push_back(sb);
  }
  if (n_fit >= (int64_t(1) << 31)) { *err = "too many local rows for 32-bit fit-row indices"; return ENKFMC_EUNSUPPORTED; }
  p->n_fit = n_fit;
  p->nnz = (int64_t)p->col.size();
  for (int64_t gi = 0; gi < n; ++gi)
    if (p->interior_src[gi] < 0) { *err = "internal: component not covered by any interior"; return ENKFMC_EINVAL; }

  // regressions grouped by the kernel that fits them (stable within a group)
  {
    const bool offsets_fit = (n + 2) * (int64_t)p->ldu < (int64_t(1) << 31);   // 32-bit offsets into U
    auto key = [&](int64_t r) {
      const int64_t pp = p->row_ptr[r + 1] - p->row_ptr[r];
      if (pp == 0) return kBucketP0;
      if (!offsets_fit || N > kBatchedMaxN || pp > kBatchedMaxP) return kBucketPlain;
      if (pp >= N) return kBucketKF;
      return (int)((pp + 15) / 16);   // p < N <= 128: 1..8 tiles
    };
    int64_t cnt[kBuckets + 1] = {};
    for (int64_t r = 0; r < n_fit; ++r) cnt[key(r) + 1]++;
    for (int b = 0; b < kBuckets; ++b) cnt[b + 1] += cnt[b];
    for (int b = 0; b <= kBuckets; ++b) p->bucket_off[b] = cnt[b];
    p->fit_rows.assign(n_fit, 0);
    int64_t fill[kBuckets];
    for (int b = 0; b < kBuckets; ++b) fill[b] = cnt[b];
    for (int64_t r = 0; r < n_fit; ++r) p->fit_rows[fill[key(r)]++] = (int32_t)r;
  }

  // local observations, per block, observation number ascending (R5: whole extended box)
  std::vector<std::vector<int32_t>> bo(p->blocks.size()), br(p->blocks.size());
  const int32_t nxy = p->nx * p->ny;
  for (int32_t o = 0; o < m; ++o) {
    const int32_t gidx = p->obs_idx[o];
    int32_t v = p->nvar - 1;
    while (v > 0 && gidx < p->var_off[v]) --v;
    const int32_t rem = gidx - p->var_off[v];
    const int32_t l = rem / nxy, lat = (rem % nxy) / p->nx, lon = rem % p->nx;
    for (int32_t k = 0; k < nsd; ++k) {
      const SubBox &sb = p->subs[k];
      if (lat < sb.ys || lat >= sb.ys + sb.BY) continue;
      int32_t ix;
      if (sb.ring) ix = lon;
      else if (p->periodic_x) ix = ((lon - sb.xs) % p->nx + p->nx) % p->nx;
      else ix = lon - sb.xs;
      if (ix < 0 || ix >= sb.BX) continue;
      const int32_t b = sb.blk0 + v;
      bo[b].push_back(o);
      br[b].push_back((l * sb.BY + (lat - sb.ys)) * sb.BX + ix);
    }
  }
  p->bobs_o.clear(); p->bobs_row.clear(); p->bobs_fit.clear(); p->ot_jmax.clear();
  p->o2b_ptr.assign(m + 1, 0);
  int64_t sumF = 0, sumS = 0, sumQ = 0;
  for (size_t b = 0; b < p->blocks.size(); ++b) {
    Block &B = p->blocks[b];
    B.obs0 = (int64_t)p->bobs_o.size();
    B.m = (int32_t)bo[b].size();
    B.nrt = (B.n + 15) / 16;
    B.ldf = (B.m + 15) / 16 * 16;
    B.F0 = sumF; B.S0 = sumS; B.Q0 = sumQ;
    sumF += (int64_t)16 * B.nrt * B.ldf; sumS += (int64_t)B.ldf * B.ldf; sumQ += (int64_t)B.ldf * N;
    p->max_bm = std::max(p->max_bm, B.m);
    // column o of F = T^-T H^T vanishes below its observed row, so each tile of
    // 16 observations is zero below the largest of its rows
    B.ot0 = (int64_t)p->ot_jmax.size();
    for (int32_t t = 0; t < B.ldf / 16; ++t) {
      int32_t jm = -1;
      for (int32_t a = 16 * t; a < std::min(B.m, 16 * t + 16); ++a) jm = std::max(jm, br[b][a]);
      p->ot_jmax.push_back(jm);
    }
    for (size_t t = 0; t < bo[b].size(); ++t) {
      p->bobs_o.push_back(bo[b][t]);
      p->bobs_row.push_back(br[b][t]);
      p->bobs_fit.push_back((int32_t)(B.row0 + br[b][t]));
      p->o2b_ptr[bo[b][t] + 1]++;
    }
  }
  p->m_local = (int64_t)p->bobs_o.size();
  p->sum_F = sumF; p->sum_S = sumS; p->sum_Q = sumQ;
  for (int32_t o = 0; o < m; ++o) p->o2b_ptr[o + 1] += p->o2b_ptr[o];
  p->o2b.assign(p->m_local, 0);
  {
    std::vector<int64_t> fill(p->o2b_ptr.begin(), p->o2b_ptr.end() - 1);
    for (int64_t t = 0; t < p->m_local; ++t) p->o2b[fill[p->bobs_o[t]]++] = (int32_t)t;
  }
  // component -> fit rows (sub-domain order), for the adjoint's halo sums
  p->g2f_ptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n_fit; ++r) p->g2f_ptr[p->fit_glob[r] + 1]++;
  for (int64_t gi = 0; gi < n; ++gi) p->g2f_ptr[gi + 1] += p->g2f_ptr[gi];
  p->g2f.assign(n_fit, 0);
  {
    std::vector<int64_t> fill(p->g2f_ptr.begin(), p->g2f_ptr.end() - 1);
    for (int64_t r = 0; r < n_fit; ++r) p->g2f[fill[p->fit_glob[r]]++] = (int32_t)r;
  }
  // transposed pattern per block: successors of each row, row ascending
  p->csc_ptr.assign(n_fit + 1, 0);
  p->csc_row.assign(p->nnz, 0);
  p->csc_nz.assign(p->nnz, 0);
  for (const Block &B : p->blocks) {
    for (int32_t i = 0; i < B.n; ++i)
      for (int64_t k = p->row_ptr[B.row0 + i]; k < p->row_ptr[B.row0 + i + 1]; ++k)
        p->csc_ptr[B.row0 + p->col[k] + 1]++;
  }
  for (int64_t r = 0; r < n_fit; ++r) p->csc_ptr[r + 1] += p->csc_ptr[r];
  {
    std::vector<int64_t> fill(p->csc_ptr.begin(), p->csc_ptr.end() - 1);
    for (const Block &B : p->blocks)
      for (int32_t i = 0; i < B.n; ++i)
        for (int64_t k = p->row_ptr[B.row0 + i]; k < p->row_ptr[B.row0 + i + 1]; ++k) {
          const int64_t slot = fill[B.row0 + p->col[k]]++;
          p->csc_row[slot] = i;
          p->csc_nz[slot] = (int32_t)(k - B.nz0);
        }
  }
  // block-sparse tiling of each block's T (16-row tiles)
  p->rt_ptr.assign(1, 0);
  p->rt_col.clear(); p->rt_slot.clear();
  p->n_rt = 0; p->n_slots = 0; p->max_rt_tiles = 0; p->max_rt_back = 0;
  for (Block &B : p->blocks) {
    B.rt0 = p->n_rt;
    for (int32_t R = 0; R < B.nrt; ++R) {
      std::vector<int32_t> cs;
      const int32_t i1 = std::min(B.n, 16 * R + 16);
      for (int32_t i = 16 * R; i < i1; ++i)
        for (int64_t k = p->row_ptr[B.row0 + i]; k < p->row_ptr[B.row0 + i + 1]; ++k)
          if (p->col[k] / 16 != R) cs.push_back(p->col[k] / 16);
      std::sort(cs.begin(), cs.end());
      cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
      for (int32_t c : cs) { p->rt_col.push_back(c); p->rt_slot.push_back((int32_t)p->n_slots++); }
      p->rt_ptr.push_back((int64_t)p->rt_col.size());
      p->max_rt_tiles = std::max(p->max_rt_tiles, (int32_t)cs.size());
      if (!cs.empty()) p->max_rt_back = std::max(p->max_rt_back, R - cs.front());
      ++p->n_rt;
    }
  }
  {
    // distances R - C of the stored tiles; the split sweeps take the first
    // contiguous run 1..d of them as near (at most 8)
    std::vector<char> seen((size_t)p->max_rt_back + 2, 0);
    for (const Block &B : p->blocks)
      for (int32_t R = 0; R < B.nrt; ++R)
        for (int64_t t = p->rt_ptr[B.rt0 + R]; t < p->rt_ptr[B.rt0 + R + 1]; ++t) seen[(size_t)(R - p->rt_col[t])] = 1;
    int32_t d = 0;
    while (d + 1 < (int32_t)seen.size() && seen[(size_t)d + 1] && d < 8) ++d;
    p->near_d = std::max(d, 1);
    // per block, the range of its distances beyond near_d
    p->far_lo = 0;
    p->far_w = 0;
    for (Block &B : p->blocks) {
      int32_t lo = 0, hi = 0;
      for (int32_t R = 0; R < B.nrt; ++R)
        for (int64_t t = p->rt_ptr[B.rt0 + R]; t < p->rt_ptr[B.rt0 + R + 1]; ++t) {
          const int32_t e = R - p->rt_col[t];
          if (e <= p->near_d) continue;
          lo = lo == 0 ? e : std::min(lo, e);
          hi = std::max(hi, e);
        }
      B.far_lo = lo;
      B.far_w = lo > 0 ? hi - lo + 1 : 0;
      if (lo > 0) p->far_lo = p->far_lo == 0 ? lo : std::min(p->far_lo, lo);
      p->far_w = std::max(p->far_w, B.far_w);
    }
    p->rt_nfar.assign((size_t)p->n_rt, 0);
    for (const Block &B : p->blocks)
      for (int32_t R = 0; R < B.nrt; ++R) {
        int32_t nf = 0;
        for (int64_t t = p->rt_ptr[B.rt0 + R]; t < p->rt_ptr[B.rt0 + R + 1]; ++t)
          if (R - p->rt_col[t] > p->near_d) ++nf;
        p->rt_nfar[(size_t)(B.rt0 + R)] = nf;
      }
  }
  if (p->n_slots >= (int64_t(1) << 31)) { *err = "too many tiles"; return ENKFMC_EUNSUPPORTED; }
  if (p->max_p > 65535) { *err = "too many predecessors"; return ENKFMC_EUNSUPPORTED; }
  p->tile_eoff.assign((size_t)16 * (p->n_slots + p->n_rt), 0);
  for (const Block &B : p->blocks)
    for (int32_t R = 0; R < B.nrt; ++R) {
      const int64_t rt = B.rt0 + R, t0 = p->rt_ptr[rt];
      const int32_t nt = (int32_t)(p->rt_ptr[rt + 1] - t0);
      for (int32_t i = 0; i < 16 && 16 * R + i < B.n; ++i) {
        const int64_t ka = p->row_ptr[B.row0 + 16 * R + i], kb = p->row_ptr[B.row0 + 16 * R + i + 1];
        int64_t k = ka;                          // tiles ascending: one pass over the row
        for (int32_t t = 0; t <= nt; ++t) {
          const int32_t C = t < nt ? p->rt_col[t0 + t] : R;
          while (k < kb && p->col[k] < 16 * C) ++k;
          p->tile_eoff[(size_t)16 * (t0 + rt + t) + i] = (uint16_t)(k - ka);
        }
        // the kernels rely on: tile t's entries are exactly those up to the
        // next tile's offset, at most 16 of them, all in columns [16C, 16C + 16)
        for (int32_t t = 0; t <= nt; ++t) {
          const int32_t C = t < nt ? p->rt_col[t0 + t] : R;
          const int64_t e0 = ka + p->tile_eoff[(size_t)16 * (t0 + rt + t) + i];
          const int64_t e1 = t < nt ? ka + p->tile_eoff[(size_t)16 * (t0 + rt + t + 1) + i] : kb;
          if (e1 < e0 || e1 - e0 > 16) { *err = "internal: tile entry ranges"; return ENKFMC_EINVAL; }
          for (int64_t k = e0; k < e1; ++k)
            if (p->col[k] < 16 * C || p->col[k] >= 16 * C + 16) { *err = "internal: tile entry ranges"; return ENKFMC_EINVAL; }
        }
        if (p->tile_eoff[(size_t)16 * (t0 + rt) + i] != 0) { *err = "internal: tile entry ranges"; return ENKFMC_EINVAL; }
      }
    }
  // transposed tile lists: for every column tile, the later row tiles (ascending)
  p->ct_ptr.assign(p->n_rt + 1, 0);
  for (const Block &B : p->blocks)
    for (int32_t R = 0; R < B.nrt; ++R)
      for (int64_t t = p->rt_ptr[B.rt0 + R]; t < p->rt_ptr[B.rt0 + R + 1]; ++t) p->ct_ptr[B.rt0 + p->rt_col[t] + 1]++;
  for (int64_t t = 0; t < p->n_rt; ++t) p->ct_ptr[t + 1] += p->ct_ptr[t];
  p->ct_row.assign(p->rt_col.size(), 0);
  p->ct_slot.assign(p->rt_col.size(), 0);
  {
    std::vector<int64_t> fill(p->ct_ptr.begin(), p->ct_ptr.end() - 1);
    for (const Block &B : p->blocks)
      for (int32_t R = 0; R < B.nrt; ++R)
        for (int64_t t = p->rt_ptr[B.rt0 + R]; t < p->rt_ptr[B.rt0 + R + 1]; ++t) {
          const int64_t slot = fill[B.rt0 + p->rt_col[t]]++;
          p->ct_row[slot] = R;
          p->ct_slot[slot] = p->rt_slot[t];
        }
  }
  p->ct_nfar.assign((size_t)p->n_rt, 0);
  for (const Block &B : p->blocks)
    for (int32_t C = 0; C < B.nrt; ++C) {
      int32_t nf = 0;
      for (int64_t t = p->ct_ptr[B.rt0 + C]; t < p->ct_ptr[B.rt0 + C + 1]; ++t)
        if (p->ct_row[t] - C > p->near_d) ++nf;
      p->ct_nfar[(size_t)(B.rt0 + C)] = nf;
    }
  compute_layout(p);
  return ENKFMC_OK;
}

void compute_layout(enkfmc_plan *p) {
  Layout &L = p->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  const size_t nb = p->blocks.size(), nf = (size_t)p->n_fit, nz = (size_t)p->nnz, n = (size_t)p->n;
  const size_t ml = (size_t)p->m_local, m = (size_t)p->m, N = (size_t)p->N;
  L.blocks = take(nb * sizeof(Block));
  L.fit_glob = take(nf * 4);
  L.fit_blk = take(nf * 4);
  L.fit_rows = take(nf * 4);
  L.row_ptr = take((nf + 1) * 8);
  L.col = take(nz * 4);
  L.csc_ptr = take((nf + 1) * 8);
  L.csc_row = take(nz * 4);
  L.csc_nz = take(nz * 4);
  L.interior_src = take(n * 4);
  L.bobs_o = take(ml * 4);
  L.bobs_row = take(ml * 4);
  L.g2f_ptr = take((n + 1) * 8);
  L.g2f = take(nf * 4);
  L.o2b_ptr = take((m + 1) * 8);
  L.o2b = take(ml * 4);
  L.bobs_fit = take(ml * 4);
  L.ot_jmax = take(p->ot_jmax.size() * 4 + 4);
  L.rt_ptr = take((size_t)(p->n_rt + 1) * 8);
  L.rt_col = take(p->rt_col.size() * 4);
  L.rt_slot = take(p->rt_slot.size() * 4);
  L.rt_nfar = take(p->rt_nfar.size() * 4 + 4);
  L.ct_nfar = take(p->ct_nfar.size() * 4 + 4);
  L.ct_ptr = take((size_t)(p->n_rt + 1) * 8);
  L.ct_row = take(p->ct_row.size() * 4);
  L.ct_slot = take(p->ct_slot.size() * 4);
  L.tile_eoff = take(p->tile_eoff.size() * 2);
  L.tval = take(nz * 8);
  L.dvec = take(nf * 8);
  L.mean = take(n * 8);
  L.U = take((n + 2) * (size_t)p->ldu * 8);   // two trailing all-zero pad rows
  L.Z = take(nf * N * 8);
  L.F = take((size_t)p->sum_F * 8);
  L.S = take((size_t)p->sum_S * 8);
  L.Q = take((size_t)p->sum_Q * 8);
  L.P = take((size_t)p->sum_Q * 8);
  L.W = take(nf * N * 8);
  L.aux1 = take(nf * N * 8);
  L.aux2 = take(nf * N * 8);
  L.aux3 = take(nz * 8);
  L.dbar = take(std::max<size_t>(nf, 256) * 8);   // also the 256 partial sums of dL/dlam and of the squared error
  L.red = take(nf * 8 + 64);
  L.tiles = take((size_t)p->n_slots * 256 * 8);
  L.tinv = take((size_t)p->n_rt * 256 * 8);
  L.tdiag = take((size_t)p->n_rt * 256 * 8);
  L.ubar = take(nf * N * 8);
  L.pcg = take((size_t)5 * nb * N * 8 + 64);   // per (block, member) scalars of the PCG + its counter
  L.status = take(64);
  L.total = off;
}

}  // namespace enkfmc
