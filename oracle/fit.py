"""Modified-Cholesky estimate of the inverse background covariance (oracle).

Test infrastructure only.

What the paper fixes
--------------------
* eq. (5): anomalies U = X_b - mean(X_b) 1^T.
* eq. (1): each component's ensemble vector is regressed on its predecessors;
  T holds the negated coefficients below a unit diagonal and D the variances of
  the regression residuals; eq. (2) / eq. (8): B^-1 ~ T^T D^-1 T.

Readings
--------
R6  The regression is solved through its (ridge) normal equations with a
    Cholesky factorisation:  G = U_P U_P^T/(N-1) + lam I,  c = U_P u/(N-1),
    beta = G^-1 c.  (The paper computes the coefficients by SVD, Section 5;
    lam = 0 gives the same least-squares solution when U_P has full row rank.)
    A Cholesky pivot <= 0 is an error (ENOTSPD), never a pseudo-inverse.
    With lam = 0 and p >= N - 1 the anomalies (rank N - 1) make G singular
    (p > N - 1) or fit u exactly (p = N - 1, D_ii = 0): both are ENOTSPD,
    decided from p and N rather than from rounding noise.
R7  D_ii = eps^T eps / (N-1) with eps = u - U_P^T beta (residual form).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import scipy.linalg as sla

from .errors import OracleError
from .geometry import Pattern


def anomalies(Xb: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """eq. (5): mean over members and centred anomalies, in float64."""
    X = np.asarray(Xb, dtype=np.float64)
    N = X.shape[1]
    mean = X.sum(axis=1) / N
    return mean, X - mean[:, None]


def fit_row(U_loc: np.ndarray, i: int, P: np.ndarray, lam: float):
    """eq. (1) for local row i with predecessor rows P (R6, R7).

    Returns (beta, d, eps).
    """
    N = U_loc.shape[1]
    u = U_loc[i]
    if P.size == 0:
        d = float(u @ u) / (N - 1)
        beta = np.zeros(0)
        eps = u.copy()
    else:
        if lam == 0.0 and P.size >= N - 1:
            raise OracleError("ENOTSPD", f"local row {i}: {P.size} predecessors need lam > 0 with N = {N}")
        UP = U_loc[P]
        G = UP @ UP.T / (N - 1) + lam * np.eye(P.size)
        c = UP @ u / (N - 1)
        try:
            L = np.linalg.cholesky(G)
        except np.linalg.LinAlgError:
            raise OracleError("ENOTSPD", f"regression Gram of local row {i} is not positive definite")
        beta = sla.cho_solve((L, True), c)
        eps = u - UP.T @ beta
        d = float(eps @ eps) / (N - 1)
    if not d > 0.0:
        raise OracleError("ENONPOS_D", f"residual variance of local row {i} is not positive")
    return beta, d, eps


def fit_row_svd(U_loc: np.ndarray, i: int, P: np.ndarray, lam: float):
    """eq. (1) for local row i by the singular value decomposition of the
    regression's design matrix, the route Section 5 proposes for accelerators.

    With A = U_P^T (N x p) = W diag(sigma) V^T (thin SVD) and mu = lam (N-1),
    the ridge solution of  min |u - A beta|^2 + mu |beta|^2  is
        beta = V diag(sigma / (sigma^2 + mu)) W^T u,
    the same beta as the normal equations of R6 (G = A^T A/(N-1) + lam I,
    c = A^T u/(N-1)).  Readings as in fit_row: lam = 0 with p >= N - 1 is
    ENOTSPD (no pseudo-inverse); D from the residual vector (R7).

    Returns (beta, d, eps).
    """
    N = U_loc.shape[1]
    u = U_loc[i]
    if P.size == 0:
        return fit_row(U_loc, i, P, lam)
    if lam == 0.0 and P.size >= N - 1:
        raise OracleError("ENOTSPD", f"local row {i}: {P.size} predecessors need lam > 0 with N = {N}")
    A = U_loc[P].T
    W, sig, Vt = np.linalg.svd(A, full_matrices=False)
    mu = lam * (N - 1)
    den = sig * sig + mu
    if not np.all(den > 0.0):
        raise OracleError("ENOTSPD", f"design matrix of local row {i} is rank deficient without a ridge")
    beta = Vt.T @ ((sig / den) * (W.T @ u))
    eps = u - A @ beta
    d = float(eps @ eps) / (N - 1)
    if not d > 0.0:
        raise OracleError("ENONPOS_D", f"residual variance of local row {i} is not positive")
    return beta, d, eps


class Factors:
    """T (strictly lower part, CSR values = -beta) and D of one sub-domain."""

    def __init__(self, pat: Pattern, tval: np.ndarray, d: np.ndarray, eps: np.ndarray):
        self.pat = pat
        self.tval = tval
        self.d = d
        self.eps = eps

    def T_dense(self) -> np.ndarray:
        n = self.pat.n_sd
        T = np.eye(n)
        for i in range(n):
            lo, hi = self.pat.row_ptr[i], self.pat.row_ptr[i + 1]
            T[i, self.pat.col_idx[lo:hi]] = self.tval[lo:hi]
        return T

    def binv_dense(self) -> np.ndarray:
        """eq. (8): T^T D^-1 T."""
        T = self.T_dense()
        return T.T @ (T / self.d[:, None])


def fit_subdomain(U: np.ndarray, pat: Pattern, lam: float, rows=None, method: str = "cholesky") -> Factors:
    """Fit every local row (or the listed ones) of one sub-domain (Alg. 3,
    first step), by the normal equations (method "cholesky", R6) or by the
    SVD of Section 5 (method "svd")."""
    row_fit = fit_row_svd if method == "svd" else fit_row
    U_loc = U[pat.loc2glob]
    n = pat.n_sd
    tval = np.zeros(pat.col_idx.shape[0])
    d = np.full(n, np.nan)
    eps = np.full((n, U.shape[1]), np.nan)
    todo = range(n) if rows is None else rows
    for i in todo:
        lo, hi = pat.row_ptr[i], pat.row_ptr[i + 1]
        beta, d[i], eps[i] = row_fit(U_loc, i, pat.col_idx[lo:hi], lam)
        tval[lo:hi] = -beta
    return Factors(pat, tval, d, eps)
