"""Assimilation cycles (oracle): perturbed observations, the cycle loop of
Alg. 1 and the RMSE of eq. (18).

Test infrastructure only.

What the paper fixes
--------------------
* Section 2.3 (after eq. 11): Y^s holds perturbed observations whose data
  errors follow N(0, R).
* Alg. 1: at every assimilation time, draw Y^s from y and R, run the analysis
  on the current background ensemble, then propagate every analysis member
  with the model to the next time.
* eq. (18), Section 4: RMSE = sqrt((1/M) sum_k (x_ref_k - x_a_k)^T
  (x_ref_k - x_a_k)) over the M assimilation times, x_a_k the analysis mean.

Readings
--------
R9  The data errors are drawn uncentred.  The paper leaves the generator to
    each processor; here it is one counter-based generator, so that a draw
    depends only on (seed, assimilation time, observation, member) and the
    oracle and the GPU draw the same numbers: Philox4x64-10 (Salmon, Moraes,
    Dror, Shaw, SC'11) with key (seed, 0) and counter (k // 4, o, cycle, 0),
    uniforms u = ((w >> 12) + 1/2) 2^-52 from its four 64-bit words, and the
    Box-Muller transform of (u_0, u_1) and (u_2, u_3) for members 4j..4j+3.
R14 eq. (18) sums over components without a 1/n; implemented as printed.
The forecast model is an input (the method does not include one).
"""
from __future__ import annotations

from typing import Callable, List, Optional, Sequence

import numpy as np

from .analysis import Result, analyze

MASK64 = (1 << 64) - 1
# Philox4x64 round multipliers and Weyl key increments of the SC'11 paper
PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def mulhilo64(a: np.ndarray, b: int):
    """High and low 64-bit halves of the 128-bit products a * b (uint64)."""
    a = np.asarray(a, np.uint64)
    lo32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    b0, b1 = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    a0, a1 = a & lo32, a >> s32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> s32) + (p01 & lo32) + (p10 & lo32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    lo = a * np.uint64(b)          # wraps modulo 2^64
    return hi, lo


def philox4x64_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x64-10 of the counters ctr (..., 4) uint64 under key (k0, k1)."""
    x = [np.array(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = (k0 + PHILOX_W[0]) & MASK64
                k1 = (k1 + PHILOX_W[1]) & MASK64
            hi0, lo0 = mulhilo64(x[0], PHILOX_M[0])
            hi1, lo1 = mulhilo64(x[2], PHILOX_M[1])
            x = [hi1 ^ x[1] ^ np.uint64(k0), lo1, hi0 ^ x[3] ^ np.uint64(k1), lo0]
    return np.stack(x, axis=-1)


def unit_open(w: np.ndarray) -> np.ndarray:
    """((w >> 12) + 1/2) 2^-52: uniforms in (0, 1), exact in float64."""
    return ((np.asarray(w, np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def box_muller(u0: np.ndarray, u1: np.ndarray):
    rho = np.sqrt(-2.0 * np.log(u0))
    return rho * np.cos(2.0 * np.pi * u1), rho * np.sin(2.0 * np.pi * u1)


def standard_normals(seed: int, cycle: int, m: int, N: int) -> np.ndarray:
    """xi[o, k] of reading R9, (m, N) float64."""
    J = (N + 3) // 4
    ctr = np.zeros((m, J, 4), np.uint64)
    ctr[..., 0] = np.arange(J, dtype=np.uint64)[None, :]
    ctr[..., 1] = np.arange(m, dtype=np.uint64)[:, None]
    ctr[..., 2] = np.uint64(int(cycle) & MASK64)
    w = philox4x64_10(ctr, (seed, 0))
    u = unit_open(w)
    z = np.empty((m, J, 4))
    z[..., 0], z[..., 1] = box_muller(u[..., 0], u[..., 1])
    z[..., 2], z[..., 3] = box_muller(u[..., 2], u[..., 3])
    return z.reshape(m, 4 * J)[:, :N]


def perturbed_observations(y: np.ndarray, r_diag: np.ndarray, seed: int, cycle: int, N: int) -> np.ndarray:
    """Y^s = y 1^T + E, E[o, k] = sqrt(r_o) xi[o, k] (Section 2.3, Alg. 1)."""
    y = np.asarray(y, np.float64)
    r = np.asarray(r_diag, np.float64)
    return y[:, None] + np.sqrt(r)[:, None] * standard_normals(seed, cycle, y.shape[0], N)


def sq_error(Xa: np.ndarray, x_ref: np.ndarray) -> float:
    """(x_ref - x_a)^T (x_ref - x_a) with x_a the analysis mean: one term of eq. (18)."""
    e = np.asarray(x_ref, np.float64) - np.asarray(Xa, np.float64).mean(axis=1)
    return float(e @ e)


def rmse(sq_errs: Sequence[float]) -> float:
    """eq. (18) from the per-time squared errors."""
    v = np.asarray(sq_errs, np.float64)
    return float(np.sqrt(v.sum() / v.size))


class Cycles:
    def __init__(self, Xa, results: List[Result], sq_err: Optional[np.ndarray], rmse_value: Optional[float]):
        self.Xa = Xa
        self.results = results
        self.sq_err = sq_err
        self.rmse = rmse_value


def assimilate(geo, Xb, observations: Sequence[np.ndarray], obs_idx, r_diag, lam, forecast: Callable, seed: int,
               x_ref: Optional[Sequence[np.ndarray]] = None, first_cycle: int = 0, keep: bool = False) -> Cycles:
    """Alg. 1 over the assimilation times of `observations`."""
    X = np.asarray(Xb, np.float64)
    N = X.shape[1]
    errs, results = [], []
    res = None
    for t, y in enumerate(observations):
        Ys = perturbed_observations(y, r_diag, seed, first_cycle + t, N)
        res = analyze(geo, X, Ys, obs_idx, r_diag, lam)
        if keep:
            results.append(res)
        if x_ref is not None:
            errs.append(sq_error(res.Xa, x_ref[t]))
        if t + 1 < len(observations):
            X = np.asarray(forecast(res.Xa), np.float64)
    if x_ref is None:
        return Cycles(res.Xa, results, None, None)
    return Cycles(res.Xa, results, np.asarray(errs), rmse(errs))
