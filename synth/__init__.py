"""Seeded synthetic inputs for the EnKF-MC hot path.

This module only draws random numbers with prescribed statistics (Gaussian
random fields, observation sites, observation noise).  It holds none of the
method's arithmetic: no regression, no analysis.  Both the FP64 CPU oracle and
the GPU path consume what it produces.

Every draw comes from ``numpy.random.Generator(PCG64(SeedSequence([160600807,
config, stream])))`` with the streams

    0 truth, 1 ensemble, 2 observation sites, 3 observation noise,
    4 perturbed-observation noise, 5 batch-instance parameters.

Fields have zero mean so that relative errors measure the increment and the
anomalies rather than an offset.

The synthetic fields stand in for the SPEEDY states of the paper's experiments
(Section 4), which are not available: the shapes (T-63 192x96 grid, several
levels and variables, ensemble size, observed fraction) follow that section.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 160600807

STREAM_TRUTH = 0
STREAM_ENSEMBLE = 1
STREAM_OBS_SITES = 2
STREAM_OBS_NOISE = 3
STREAM_PERTURB = 4
STREAM_INSTANCES = 5


def rng(config: int, stream: int, extra: int = 0) -> np.random.Generator:
    """Counter-keyed generator for (config, stream[, extra])."""
    key = [SEED_BASE, int(config), int(stream)]
    if extra:
        key.append(int(extra))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(key)))


@dataclass
class Problem:
    """One EnKF-MC assimilation problem: geometry, ensemble and observations.

    geometry keys: nx, ny, nvar, nlev (list), periodic_x, sdx, sdy, r_h, r_v.
    Xb is (n, N) row-major (component rows, members contiguous).
    """

    name: str
    geometry: Dict
    N: int
    Xb: np.ndarray            # (n, N), float32 or float64
    x_true: np.ndarray        # (n,), float64
    obs_idx: np.ndarray       # (m,), int32, strictly increasing
    r_diag: np.ndarray        # (m,), float64 > 0
    Y: np.ndarray             # (m, N), float64 perturbed observations
    ridge: float
    meta: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.Xb.shape[0])

    @property
    def m(self) -> int:
        return int(self.obs_idx.shape[0])


def geometry(nx, ny, nlev, periodic_x=True, sdx=1, sdy=1, r_h=1, r_v=0) -> Dict:
    nlev = [int(v) for v in nlev]
    return dict(nx=int(nx), ny=int(ny), nvar=len(nlev), nlev=nlev, periodic_x=int(bool(periodic_x)),
                sdx=int(sdx), sdy=int(sdy), r_h=int(r_h), r_v=int(r_v))


def state_size(geo: Dict) -> int:
    return geo["nx"] * geo["ny"] * int(sum(geo["nlev"]))


# ----------------------------------------------------------------------------
# Gaussian random fields
# ----------------------------------------------------------------------------

def _dense_corr_2d(nx: int, ny: int, L: float, periodic_x: bool) -> np.ndarray:
    """exp(-d/L) over an nx*ny grid (lon fastest), Euclidean cell distance,
    longitude wrapped when periodic_x."""
    x = np.tile(np.arange(nx), ny).astype(np.float64)
    y = np.repeat(np.arange(ny), nx).astype(np.float64)
    dx = np.abs(x[:, None] - x[None, :])
    if periodic_x:
        dx = np.minimum(dx, nx - dx)
    dy = y[:, None] - y[None, :]
    return np.exp(-np.sqrt(dx * dx + dy * dy) / L)


def _ring_corr(n: int, L: float) -> np.ndarray:
    i = np.arange(n, dtype=np.float64)
    d = np.abs(i[:, None] - i[None, :])
    d = np.minimum(d, n - d)
    return np.exp(-d / L)


def _chol_with_jitter(S: np.ndarray) -> np.ndarray:
    jitter = 0.0
    for _ in range(12):
        try:
            return np.linalg.cholesky(S + jitter * np.eye(S.shape[0]))
        except np.linalg.LinAlgError:
            jitter = 1e-10 if jitter == 0.0 else jitter * 10.0
    raise np.linalg.LinAlgError("correlation matrix not positive definite even with jitter")


def dense_grf(geo: Dict, L_h: float, L_v: float, count: int, g: np.random.Generator) -> np.ndarray:
    """count independent zero-mean unit-variance fields, returned (n, count).

    Per variable: horizontal exp(-d/L_h) (dense Cholesky), vertical exact
    exponential correlation exp(-|dl|/L_v) through an AR(1) recursion.
    """
    nx, ny = geo["nx"], geo["ny"]
    if ny == 1 and geo["periodic_x"]:
        Lh = _chol_with_jitter(_ring_corr(nx, L_h))
    else:
        Lh = _chol_with_jitter(_dense_corr_2d(nx, ny, L_h, bool(geo["periodic_x"])))
    rho = float(np.exp(-1.0 / L_v)) if L_v > 0 else 0.0
    out = []
    for nlev in geo["nlev"]:
        prev = None
        for _lev in range(nlev):
            xi = Lh @ g.standard_normal((nx * ny, count))
            cur = xi if prev is None else rho * prev + np.sqrt(1.0 - rho * rho) * xi
            out.append(cur)
            prev = cur
    return np.concatenate(out, axis=0)


def fft_grf_2d(nx: int, ny: int, L: float, count: int, g: np.random.Generator, meta: Optional[Dict] = None) -> np.ndarray:
    """count fields (count, ny, nx) with exp(-d/L) correlation by circulant
    embedding on an nx x (2*ny) torus, cropped to ny latitudes."""
    my = 2 * ny
    ix = np.arange(nx)
    iy = np.arange(my)
    dx = np.minimum(ix, nx - ix).astype(np.float64)
    dy = np.minimum(iy, my - iy).astype(np.float64)
    c = np.exp(-np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2) / L)
    lam = np.real(np.fft.fft2(c))
    neg = int(np.sum(lam < 0))
    if meta is not None:
        meta["clipped_eigenvalues"] = meta.get("clipped_eigenvalues", 0) + neg
    lam = np.sqrt(np.maximum(lam, 0.0) / (nx * my))
    out = np.empty((count, ny, nx), dtype=np.float64)
    k = 0
    while k < count:
        e = g.standard_normal((my, nx)) + 1j * g.standard_normal((my, nx))
        f = np.fft.fft2(lam * e)
        out[k] = f.real[:ny]
        k += 1
        if k < count:
            out[k] = f.imag[:ny]
            k += 1
    return out


def fft_grf(geo: Dict, L_h: float, L_v: float, count: int, g: np.random.Generator, meta: Optional[Dict] = None,
            dtype=np.float64) -> np.ndarray:
    """(n, count) fields: per variable, per level FFT GRF, AR(1) in the vertical."""
    nx, ny = geo["nx"], geo["ny"]
    rho = float(np.exp(-1.0 / L_v)) if L_v > 0 else 0.0
    n = state_size(geo)
    out = np.empty((n, count), dtype=dtype)
    row = 0
    for nlev in geo["nlev"]:
        prev = None
        for _lev in range(nlev):
            xi = fft_grf_2d(nx, ny, L_h, count, g, meta).reshape(count, nx * ny).T
            cur = xi if prev is None else rho * prev + np.sqrt(1.0 - rho * rho) * xi
            out[row:row + nx * ny] = cur
            row += nx * ny
            prev = cur
    return out


# ----------------------------------------------------------------------------
# Observations
# ----------------------------------------------------------------------------

def observe(x_true: np.ndarray, obs_idx: np.ndarray, r_diag: np.ndarray, N: int,
            g_noise: np.random.Generator, g_pert: np.random.Generator) -> np.ndarray:
    """Perturbed observations: y = x_true[obs] + e, e ~ N(0, R); Y[:, c] = y + e_c, e_c ~ N(0, R)."""
    sd = np.sqrt(r_diag)
    y = x_true[obs_idx] + sd * g_noise.standard_normal(obs_idx.shape[0])
    return y[:, None] + sd[:, None] * g_pert.standard_normal((obs_idx.shape[0], N))


def random_sites(n: int, m: int, g: np.random.Generator) -> np.ndarray:
    return np.sort(g.choice(n, size=m, replace=False)).astype(np.int32)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def make_ring(n=40, N=20, r=2, L=4.0, obs_stride=2, R=0.01, ridge=0.0, config=1) -> Problem:
    """1-D periodic state, one sub-domain (the 40-component ring workload)."""
    geo = geometry(n, 1, [1], periodic_x=True, sdx=1, sdy=1, r_h=r, r_v=0)
    S = _chol_with_jitter(_ring_corr(n, L))
    x_true = S @ rng(config, STREAM_TRUTH).standard_normal(n)
    Xb = S @ rng(config, STREAM_ENSEMBLE).standard_normal((n, N))
    obs_idx = np.arange(0, n, obs_stride, dtype=np.int32)
    r_diag = np.full(obs_idx.shape[0], R)
    Y = observe(x_true, obs_idx, r_diag, N, rng(config, STREAM_OBS_NOISE), rng(config, STREAM_PERTURB))
    return Problem("ring40", geo, N, Xb, x_true, obs_idx, r_diag, Y, ridge)


def make_grid2d(nx=96, ny=48, N=40, r=3, L=3.0, sdx=8, sdy=4, obs_frac=0.25, R=0.05, ridge=0.0,
                config=2, dtype=np.float64) -> Problem:
    """2-D single-level lon-lat grid, dense exponential GRF, sdx x sdy tiles."""
    geo = geometry(nx, ny, [1], periodic_x=True, sdx=sdx, sdy=sdy, r_h=r, r_v=0)
    n = nx * ny
    S = _chol_with_jitter(_dense_corr_2d(nx, ny, L, True))
    x_true = S @ rng(config, STREAM_TRUTH).standard_normal(n)
    Xb = (S @ rng(config, STREAM_ENSEMBLE).standard_normal((n, N))).astype(dtype)
    m = int(round(obs_frac * n))
    obs_idx = random_sites(n, m, rng(config, STREAM_OBS_SITES))
    r_diag = np.full(m, R)
    Y = observe(x_true, obs_idx, r_diag, N, rng(config, STREAM_OBS_NOISE), rng(config, STREAM_PERTURB))
    return Problem(f"grid{nx}x{ny}", geo, N, Xb, x_true, obs_idx, r_diag, Y, ridge)


T63_VARS = ("u", "v", "T", "q", "ps")
T63_R = {"u": 0.04, "v": 0.04, "T": 0.02, "q": 0.08, "ps": 0.01}


def make_t63(N=80, nx=192, ny=96, levels=7, r_h=4, r_v=1, L_h=4.0, L_v=1.0, sdx=24, sdy=12,
             obs_frac=0.05, ridge=1e-3, config=3, dtype=np.float32) -> Problem:
    """T-63-shaped state: 192x96 grid, 7 levels of u, v, T, q plus surface
    pressure; per-variable unit-variance GRF (FFT circulant embedding)."""
    nlev = [levels] * 4 + [1]
    geo = geometry(nx, ny, nlev, periodic_x=True, sdx=sdx, sdy=sdy, r_h=r_h, r_v=r_v)
    n = state_size(geo)
    meta: Dict = {}
    x_true = fft_grf(geo, L_h, L_v, 1, rng(config, STREAM_TRUTH), meta)[:, 0]
    Xb = fft_grf(geo, L_h, L_v, N, rng(config, STREAM_ENSEMBLE), meta, dtype=dtype)
    m = int(round(obs_frac * n))
    obs_idx = random_sites(n, m, rng(config, STREAM_OBS_SITES))
    var_of_row = np.repeat(np.arange(5), [nx * ny * L for L in nlev])
    r_by_var = np.array([T63_R[v] for v in T63_VARS])
    r_diag = r_by_var[var_of_row[obs_idx]]
    Y = observe(x_true, obs_idx, r_diag, N, rng(config, STREAM_OBS_NOISE), rng(config, STREAM_PERTURB))
    return Problem(f"t63_{nx}x{ny}x{levels}", geo, N, Xb, x_true, obs_idx, r_diag, Y, ridge, meta)


def make_small(nx=12, ny=8, nlev=(2,), N=16, r_h=1, r_v=1, L_h=2.0, L_v=1.0, sdx=2, sdy=2, periodic_x=True,
               obs_frac=0.3, R=0.05, ridge=0.0, config=100, dtype=np.float64, name="small") -> Problem:
    """Small dense-GRF problem for tests (n up to a few thousand)."""
    geo = geometry(nx, ny, list(nlev), periodic_x=periodic_x, sdx=sdx, sdy=sdy, r_h=r_h, r_v=r_v)
    n = state_size(geo)
    x_true = dense_grf(geo, L_h, L_v, 1, rng(config, STREAM_TRUTH))[:, 0]
    Xb = dense_grf(geo, L_h, L_v, N, rng(config, STREAM_ENSEMBLE)).astype(dtype)
    m = int(round(obs_frac * n))
    obs_idx = random_sites(n, m, rng(config, STREAM_OBS_SITES)) if m > 0 else np.zeros(0, np.int32)
    r_diag = np.full(m, R)
    Y = observe(x_true, obs_idx, r_diag, N, rng(config, STREAM_OBS_NOISE), rng(config, STREAM_PERTURB))
    return Problem(name, geo, N, Xb, x_true, obs_idx, r_diag, Y, ridge)


def linear_forecast(X: np.ndarray, geo: Dict, shift: int = 1) -> np.ndarray:
    """Synthetic forecast: zonal shift of every level by `shift` cells (exact, linear)."""
    nx, ny = geo["nx"], geo["ny"]
    nl = int(sum(geo["nlev"]))
    tail = X.shape[1:]
    Xr = X.reshape((nl, ny, nx) + tail)
    return np.roll(Xr, shift, axis=2).reshape(X.shape)


def instance_params(count: int = 64, config: int = 5) -> List[Dict]:
    """Parameters of an uneven batch of single-variable instances."""
    g = rng(config, STREAM_INSTANCES)
    shapes = [(32, 16), (48, 24), (64, 32), (96, 48), (128, 64), (192, 96)]
    out = []
    for k in range(count):
        nx, ny = shapes[int(g.integers(0, len(shapes)))]
        lev = int(g.integers(1, 8))
        out.append(dict(nx=nx, ny=ny, nlev=lev, N=int(g.integers(20, 121)), r=int(g.integers(1, 6)),
                        r_v=1 if lev > 1 else 0, obs_frac=float(g.uniform(0.02, 0.30)), R=0.05, ridge=1e-3,
                        sdx=nx // 8, sdy=ny // 8, seed=k))
    return out


def make_instance(k: int, params: Optional[List[Dict]] = None, L_h: float = 3.0, L_v: float = 1.0, config: int = 5,
                  dtype=np.float64) -> Problem:
    """Instance k of the uneven batch: one variable on its own grid, FFT GRF
    fields, observation sites and noise from streams seeded with (config, k)."""
    d = (params or instance_params(config=config))[k]
    geo = geometry(d["nx"], d["ny"], [d["nlev"]], periodic_x=True, sdx=d["sdx"], sdy=d["sdy"], r_h=d["r"],
                   r_v=d["r_v"])
    n = state_size(geo)
    x_true = fft_grf(geo, L_h, L_v, 1, rng(config, STREAM_TRUTH, k))[:, 0]
    Xb = fft_grf(geo, L_h, L_v, d["N"], rng(config, STREAM_ENSEMBLE, k), dtype=dtype)
    m = int(round(d["obs_frac"] * n))
    obs_idx = random_sites(n, m, rng(config, STREAM_OBS_SITES, k))
    r_diag = np.full(m, d["R"])
    Y = observe(x_true, obs_idx, r_diag, d["N"], rng(config, STREAM_OBS_NOISE, k), rng(config, STREAM_PERTURB, k))
    return Problem(f"instance{k}", geo, d["N"], Xb, x_true, obs_idx, r_diag, Y, d["ridge"])


def cycle_observations(p: Problem, cycles: int, shift: int = 1, config: int = 4) -> List[tuple]:
    """Truth and perturbed observations of `cycles` assimilation cycles: the
    truth of cycle t is the synthetic forecast applied t times to p.x_true
    (cycle 0 is p's own), observed at p's fixed sites with fresh noise."""
    out = [(np.asarray(p.x_true, np.float64), p.Y)]
    x = np.asarray(p.x_true, np.float64)
    for t in range(1, cycles):
        x = linear_forecast(x, p.geometry, shift)
        Y = observe(x, p.obs_idx, p.r_diag, p.N, rng(config, STREAM_OBS_NOISE, t), rng(config, STREAM_PERTURB, t))
        out.append((x, Y))
    return out


def cycle_truth_and_obs(p: Problem, cycles: int, shift: int = 1, config: int = 4) -> List[tuple]:
    """Truth x_t and unperturbed observations y_t = x_t[obs] + e_t, e_t ~ N(0, R),
    of `cycles` assimilation times: x_t is the synthetic forecast applied t
    times to p.x_true.  The perturbation of y_t into Y^s is left to the method."""
    out = []
    x = np.asarray(p.x_true, np.float64)
    sd = np.sqrt(p.r_diag)
    for t in range(cycles):
        if t > 0:
            x = linear_forecast(x, p.geometry, shift)
        y = x[p.obs_idx] + sd * rng(config, STREAM_OBS_NOISE, 1000 + t).standard_normal(p.obs_idx.shape[0])
        out.append((x, y))
    return out

