"""Sub-domain decomposition and radius-restricted predecessors (oracle).

Test infrastructure only.

What the paper fixes
--------------------
* Section 3: the domain is split into Delta sub-domains; each sub-domain adds
  boundary (halo) points so that its local estimate of B^-1 sees the
  neighbourhood of its border points; after the local analysis the boundary
  points are discarded and only the sub-domain's own points are mapped back
  (eq. 14 and the text that follows it; Alg. 2 decomposition and merge steps).
* Section 2.3 (text after eq. 9, Fig. 2): the predecessors of a component are
  restricted to the components inside its local box of radius r that come
  before it in the labelling.
* Section 2.2: the local box of radius r is (2r+1) x (2r+1) grid points.

Readings (where the paper is silent, ambiguous or self-contradictory)
--------------------------------------------------------------------
R1  Global ordering: variable-major, then level, then latitude, then longitude
    (longitude fastest).  The text after eq. 9 says row-major; the Fig. 2
    caption says column-major.
R2  Local box: L-infinity box of half-width r_h in longitude and latitude and
    r_v in levels.
R3  No predecessors across variables (B^-1 block-diagonal per variable).
R4  Halo: rectangular, width r_h in longitude and latitude, all levels;
    clipped at the poles, wrapped in longitude when the grid is periodic.
    Tiles: floor split, the remainder goes to the first tiles.
R5  An observation belongs to every sub-domain whose extended box holds it.
R10 "Comes before" is judged in the sub-domain's local order (the local
    assimilation only sees local data), which differs from the global order
    at the periodic seam.
R12 One tile in longitude on a periodic grid (the ring): no longitude halo, and
    longitude distance is periodic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List

import numpy as np

from .errors import OracleError


def tile_bounds(extent: int, tiles: int, k: int):
    """[start, end) of tile k when `extent` cells are split into `tiles` (R4)."""
    base, rem = divmod(extent, tiles)
    start = k * base + min(k, rem)
    return start, start + base + (1 if k < rem else 0)


@dataclass
class Box:
    """Extended box of one sub-domain."""
    k: int
    kx: int
    ky: int
    x0: int          # interior lon [x0, x1)
    x1: int
    y0: int          # interior lat [y0, y1)
    y1: int
    xs: int          # global lon of local lon 0 (may be negative before wrapping)
    BX: int
    ys: int
    BY: int
    ring: bool

    def glon(self, ix: int, nx: int) -> int:
        return (self.xs + ix) % nx

    def glat(self, iy: int) -> int:
        return self.ys + iy


def validate(geo: Dict) -> None:
    nx, ny, sdx, sdy = geo["nx"], geo["ny"], geo["sdx"], geo["sdy"]
    if nx < 1 or ny < 1 or sdx < 1 or sdy < 1 or sdx > nx or sdy > ny:
        raise OracleError("EINVAL", "bad grid or tile counts")
    if geo["r_h"] < 0 or geo["r_v"] < 0 or len(geo["nlev"]) != geo["nvar"] or min(geo["nlev"]) < 1:
        raise OracleError("EINVAL", "bad radius or levels")
    if geo["periodic_x"] and sdx > 1:
        widest = tile_bounds(nx, sdx, 0)[1] - tile_bounds(nx, sdx, 0)[0]
        if widest + 2 * geo["r_h"] > nx:
            raise OracleError("EINVAL", "longitude halo wraps onto its own tile")


def box(geo: Dict, k: int) -> Box:
    """Extended box of sub-domain k = ky * sdx + kx (R4, R12)."""
    nx, ny, sdx, r = geo["nx"], geo["ny"], geo["sdx"], geo["r_h"]
    if not 0 <= k < sdx * geo["sdy"]:
        raise OracleError("EINVAL", f"sub-domain {k} outside 0..{sdx * geo['sdy'] - 1}")
    kx, ky = k % sdx, k // sdx
    x0, x1 = tile_bounds(nx, sdx, kx)
    y0, y1 = tile_bounds(ny, geo["sdy"], ky)
    ring = bool(geo["periodic_x"]) and sdx == 1
    if ring:
        xs, BX = 0, nx
    elif geo["periodic_x"]:
        xs, BX = x0 - r, (x1 - x0) + 2 * r
    else:
        xs = max(0, x0 - r)
        BX = min(nx, x1 + r) - xs
    ys = max(0, y0 - r)
    BY = min(ny, y1 + r) - ys
    return Box(k, kx, ky, x0, x1, y0, y1, xs, BX, ys, BY, ring)


def n_subdomains(geo: Dict) -> int:
    return geo["sdx"] * geo["sdy"]


def global_index(geo: Dict, v: int, lev: int, lat: int, lon: int) -> int:
    """R1: variable-major, level, latitude, longitude."""
    nx, ny = geo["nx"], geo["ny"]
    off = nx * ny * int(sum(geo["nlev"][:v]))
    return off + (lev * ny + lat) * nx + lon


def local_coords(geo: Dict, b: Box) -> List[tuple]:
    """(v, lev, iy, ix) of every local row, in local order (R1 applied to the box)."""
    out = []
    for v in range(geo["nvar"]):
        for lev in range(geo["nlev"][v]):
            for iy in range(b.BY):
                for ix in range(b.BX):
                    out.append((v, lev, iy, ix))
    return out


def lon_distance(b: Box, nx: int, ix: int, jx: int) -> int:
    d = abs(ix - jx)
    return min(d, nx - d) if b.ring else d


def predecessors(geo: Dict, b: Box, coords: List[tuple], index_of: Dict[tuple, int], i: int) -> List[int]:
    """Local rows that precede row i in local order and lie in its local box
    (R2, R3, R10, R12).  Enumerates the box around row i, keeps lower indices."""
    v, lev, iy, ix = coords[i]
    r, rv, nx = geo["r_h"], geo["r_v"], geo["nx"]
    out = []
    for lev2 in range(max(0, lev - rv), min(geo["nlev"][v], lev + rv + 1)):
        for iy2 in range(max(0, iy - r), min(b.BY, iy + r + 1)):
            for ix2 in range(b.BX):
                if lon_distance(b, nx, ix, ix2) > r:
                    continue
                j = index_of[(v, lev2, iy2, ix2)]
                if j < i:
                    out.append(j)
    return sorted(out)


@dataclass
class Pattern:
    """Everything the decomposition fixes for one sub-domain."""
    box: Box
    coords: List[tuple]
    loc2glob: np.ndarray      # (n_sd,) int64
    interior: np.ndarray      # (n_sd,) bool
    row_ptr: np.ndarray       # (n_sd+1,) int64
    col_idx: np.ndarray       # (nnz,) int64, ascending within a row
    obs: np.ndarray           # (m_sd,) global observation numbers o, ascending
    obs_row: np.ndarray       # (m_sd,) local row of each local observation

    @property
    def n_sd(self) -> int:
        return int(self.loc2glob.shape[0])

    def preds(self, i: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[i]:self.row_ptr[i + 1]]


def subdomain_pattern(geo: Dict, k: int, obs_idx: np.ndarray, rows=None) -> Pattern:
    """Decomposition of sub-domain k (Alg. 2 decomposition step).

    rows: optional subset of local rows whose predecessor lists are needed;
    the others get empty lists (used to sample very large sub-domains).
    """
    validate(geo)
    b = box(geo, k)
    nx = geo["nx"]
    coords = local_coords(geo, b)
    index_of = {c: i for i, c in enumerate(coords)}
    loc2glob = np.array([global_index(geo, v, lev, b.glat(iy), b.glon(ix, nx)) for (v, lev, iy, ix) in coords],
                        dtype=np.int64)
    interior = np.array([(b.x0 <= (b.xs + ix) < b.x1 or (b.ring)) and b.y0 <= b.glat(iy) < b.y1
                         for (v, lev, iy, ix) in coords], dtype=bool)
    want = set(range(len(coords))) if rows is None else set(int(i) for i in rows)
    row_ptr = [0]
    cols: List[int] = []
    for i in range(len(coords)):
        if i in want:
            cols.extend(predecessors(geo, b, coords, index_of, i))
        row_ptr.append(len(cols))
    glob2loc = {int(g): i for i, g in enumerate(loc2glob)}
    obs, obs_row = [], []
    for o, g in enumerate(np.asarray(obs_idx).tolist()):
        if g in glob2loc:
            obs.append(o)
            obs_row.append(glob2loc[g])
    return Pattern(b, coords, loc2glob, interior, np.array(row_ptr, np.int64), np.array(cols, np.int64),
                   np.array(obs, np.int64), np.array(obs_row, np.int64))


def all_patterns(geo: Dict, obs_idx: np.ndarray) -> List[Pattern]:
    return [subdomain_pattern(geo, k, obs_idx) for k in range(n_subdomains(geo))]


def check_obs(n: int, obs_idx: np.ndarray) -> None:
    o = np.asarray(obs_idx)
    if o.size and (o.min() < 0 or o.max() >= n or np.any(np.diff(o) <= 0)):
        raise OracleError("EINVAL", "obs_idx must be strictly increasing and inside [0, n)")
