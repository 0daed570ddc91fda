"""Local analysis and map-back (oracle).

Test infrastructure only.

What the paper fixes
--------------------
* eq. (10): X_a = X_b + dX.
* eq. (11), primal form: dX = [B^-1 + H^T R^-1 H]^-1 H^T R^-1 [Y^s - H X_b],
  with B^-1 = T^T D^-1 T from the local fit (eq. 8).
* Alg. 3: each sub-domain estimates its own B^-1 from its local ensemble and
  solves the local primal system with its local observations.
* Alg. 2 merge step and the text after eq. 14: boundary rows are discarded,
  interior rows are written back; sub-domains' interiors do not intersect.
* eqs. (12)-(13), dual form: dX = X V^T [R + V V^T]^-1 [Y^s - H X_b] with
  T X = D^{1/2} and V = H X (used here only as an independent cross-check).

Readings
--------
R8  eq. (14) and Alg. 3 as printed drop an inverse and a factor H^T R^-1; the
    oracle solves eq. (11) per sub-domain with the local arrays.
R9  Y^s (perturbed observations) is an input.
The local system is solved directly (dense Cholesky).  Because T has no
cross-variable entries (R3), H selects components and R is diagonal, the local
matrix is block-diagonal per variable; each variable block is solved on its
own, which is the same linear system.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .fit import Factors, anomalies, fit_subdomain
from .geometry import Pattern, all_patterns, check_obs


def var_blocks(pat: Pattern):
    """Contiguous local-row ranges [lo, hi) of each variable."""
    vs = np.array([c[0] for c in pat.coords])
    out = []
    for v in np.unique(vs):
        idx = np.nonzero(vs == v)[0]
        out.append((int(v), int(idx[0]), int(idx[-1]) + 1))
    return out


def innovations(Xb: np.ndarray, Y: np.ndarray, obs_idx: np.ndarray, pat: Pattern) -> np.ndarray:
    """Y^s - H X_b for the sub-domain's observations (m_sd x N)."""
    X = np.asarray(Xb, dtype=np.float64)
    return np.asarray(Y, np.float64)[pat.obs] - X[np.asarray(obs_idx)[pat.obs]]


def block_T(fac: Factors, lo: int, hi: int) -> np.ndarray:
    """Dense unit-lower T restricted to local rows/cols [lo, hi)."""
    pat = fac.pat
    T = np.eye(hi - lo)
    for i in range(lo, hi):
        a, b = pat.row_ptr[i], pat.row_ptr[i + 1]
        cols = pat.col_idx[a:b]
        T[i - lo, cols - lo] = fac.tval[a:b]
    return T


def block_system(fac: Factors, lo: int, hi: int, r_diag: np.ndarray):
    """A = T^T D^-1 T + H^T R^-1 H on rows [lo, hi) and the local obs inside them."""
    pat = fac.pat
    T = block_T(fac, lo, hi)
    A = T.T @ (T / fac.d[lo:hi, None])
    sel = np.nonzero((pat.obs_row >= lo) & (pat.obs_row < hi))[0]
    rows = pat.obs_row[sel] - lo
    rv = np.asarray(r_diag, np.float64)[pat.obs[sel]]
    A[rows, rows] += 1.0 / rv
    return A, sel, rows, rv


def solve_block(fac: Factors, lo: int, hi: int, innov: np.ndarray, r_diag: np.ndarray) -> np.ndarray:
    """Z = A^-1 H^T R^-1 (Y^s - H X_b) on one variable block (eq. 11)."""
    A, sel, rows, rv = block_system(fac, lo, hi, r_diag)
    N = innov.shape[1]
    B = np.zeros((hi - lo, N))
    B[rows] = innov[sel] / rv[:, None]
    if sel.size == 0:
        return B
    return sla.cho_solve(sla.cho_factor(A, lower=True), B)


def solve_subdomain(fac: Factors, innov: np.ndarray, r_diag: np.ndarray) -> np.ndarray:
    """Local increment Z (n_sd x N) of one sub-domain, block by block."""
    Z = np.zeros((fac.pat.n_sd, innov.shape[1]))
    for _v, lo, hi in var_blocks(fac.pat):
        Z[lo:hi] = solve_block(fac, lo, hi, innov, r_diag)
    return Z


def solve_subdomain_dense(fac: Factors, innov: np.ndarray, r_diag: np.ndarray) -> np.ndarray:
    """Same increment from the whole local matrix at once (for small cases)."""
    n = fac.pat.n_sd
    A, sel, rows, rv = block_system(fac, 0, n, r_diag)
    B = np.zeros((n, innov.shape[1]))
    B[rows] = innov[sel] / rv[:, None]
    return np.linalg.solve(A, B)


def dual_increment(fac: Factors, lo: int, hi: int, innov: np.ndarray, r_diag: np.ndarray) -> np.ndarray:
    """eqs. (12)-(13) on one variable block: T X = D^{1/2}, V = H X,
    dX = X V^T (R + V V^T)^-1 (Y^s - H X_b)."""
    pat = fac.pat
    T = block_T(fac, lo, hi)
    Xs = sla.solve_triangular(T, np.diag(np.sqrt(fac.d[lo:hi])), lower=True, unit_diagonal=True)
    sel = np.nonzero((pat.obs_row >= lo) & (pat.obs_row < hi))[0]
    rows = pat.obs_row[sel] - lo
    if sel.size == 0:
        return np.zeros((hi - lo, innov.shape[1]))
    V = Xs[rows]
    S = np.diag(np.asarray(r_diag, np.float64)[pat.obs[sel]]) + V @ V.T
    return Xs @ (V.T @ np.linalg.solve(S, innov[sel]))


class Result:
    def __init__(self, Xa, patterns, factors, Z, innov, mean, U):
        self.Xa = Xa
        self.patterns = patterns
        self.factors = factors
        self.Z = Z
        self.innov = innov
        self.mean = mean
        self.U = U


def analyze(geo, Xb, Y, obs_idx, r_diag, lam, patterns: Optional[List[Pattern]] = None) -> Result:
    """Alg. 2: decompose, fit and solve every sub-domain, merge interiors."""
    X = np.asarray(Xb, np.float64)
    check_obs(X.shape[0], obs_idx)
    if patterns is None:
        patterns = all_patterns(geo, obs_idx)
    mean, U = anomalies(X)
    Xa = np.full_like(X, np.nan)
    factors, Zs, innovs = [], [], []
    for pat in patterns:
        fac = fit_subdomain(U, pat, lam)
        innov = innovations(X, Y, obs_idx, pat)
        Z = solve_subdomain(fac, innov, r_diag)
        inner = pat.interior
        Xa[pat.loc2glob[inner]] = X[pat.loc2glob[inner]] + Z[inner]
        factors.append(fac)
        Zs.append(Z)
        innovs.append(innov)
    return Result(Xa, patterns, factors, Zs, innovs, mean, U)


def rmse(x_ref: np.ndarray, x_a: np.ndarray) -> float:
    """eq. (18) for one assimilation time (sum over components, no 1/n; R14)."""
    e = np.asarray(x_ref, np.float64) - np.asarray(x_a, np.float64)
    return float(np.sqrt(e @ e))
