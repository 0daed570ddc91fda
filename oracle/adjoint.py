"""Reverse-mode derivative of fit + local analysis (oracle).

Test infrastructure only.  Given Gbar = dL/dX_a it returns dL/dX_b,
dL/dlog(r) (r = diag R) and dL/dlam (the ridge of the regressions).

Derivation (forward definitions in fit.py and analysis.py):
  per sub-domain and variable block   A Z = B,  A = T^T D^-1 T + H^T R^-1 H,
  B rows at observations = (Y^s - X_b[obs]) / r,   X_a = X_b + Z on interior rows.

  Zbar   = Gbar on interior rows, 0 on boundary rows
  W      = A^-1 Zbar                           (A symmetric)
  Abar   = -W Z^T,   Bbar = W
  r:     dlog r_o += (1/r_o) sum_c W_jc (Z_jc - innov_oc)          (j = local row of o)
  X_b:   dX_b[obs_o] -= W_j / r_o ;  dX_b += Gbar (direct term)
  T, D:  Tbar = D^-1 T (Abar + Abar^T)  ->  Tbar_iq = -sum_c [(D^-1 T W)_ic Z_qc + (D^-1 T Z)_ic W_qc]
         Dbar_i = d_i^-2 sum_c (T W)_ic (T Z)_ic
  regression of row i (beta = -T_{i,P}, d_i = eps^T eps/(N-1), G beta = c):
         epsbar = 2 Dbar_i eps/(N-1);  betabar = -Tbar_{i,P} - U_P epsbar
         s = G^-1 betabar;  lambar -= s.beta
         Ubar_P += [s u_i^T - (s beta^T + beta s^T) U_P]/(N-1) - beta epsbar^T
         ubar_i += U_P^T s/(N-1) + epsbar
  anomalies (eq. 5): dX_b += Ubar - mean_over_members(Ubar)
Contributions of overlapping boundary rows are summed over sub-domains in
sub-domain order.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .analysis import Result, block_T, block_system, var_blocks


def analyze_backward(Xb, obs_idx, r_diag, lam, res: Result, Gbar: np.ndarray):
    X = np.asarray(Xb, np.float64)
    Gbar = np.asarray(Gbar, np.float64)
    n, N = X.shape
    r_diag = np.asarray(r_diag, np.float64)
    obs_idx = np.asarray(obs_idx)
    dXb = Gbar.copy()
    dlogR = np.zeros(r_diag.shape[0])
    dlam = 0.0
    Ubar = np.zeros((n, N))
    U = res.U
    for pat, fac, Z, innov in zip(res.patterns, res.factors, res.Z, res.innov):
        U_loc = U[pat.loc2glob]
        Ubar_loc = np.zeros_like(U_loc)
        Zbar = np.zeros_like(Z)
        Zbar[pat.interior] = Gbar[pat.loc2glob[pat.interior]]
        for _v, lo, hi in var_blocks(pat):
            A, sel, rows, rv = block_system(fac, lo, hi, r_diag)
            W = sla.cho_solve(sla.cho_factor(A, lower=True), Zbar[lo:hi])
            Zb = Z[lo:hi]
            for s_, j, r_o in zip(sel, rows, rv):
                o = pat.obs[s_]
                dlogR[o] += float(W[j] @ (Zb[j] - innov[s_])) / r_o
                dXb[obs_idx[o]] -= W[j] / r_o
            T = block_T(fac, lo, hi)
            TZ = T @ Zb
            TW = T @ W
            d = fac.d[lo:hi]
            Dbar = np.einsum("ic,ic->i", TW, TZ) / (d * d)
            for i in range(lo, hi):
                a, b = pat.row_ptr[i], pat.row_ptr[i + 1]
                P = pat.col_idx[a:b]
                ii = i - lo
                eps = fac.eps[i]
                epsbar = 2.0 * Dbar[ii] * eps / (N - 1)
                Ubar_loc[i] += epsbar
                if P.size == 0:
                    continue
                Pl = P - lo
                Tbar =-(Zb[Pl] @ (TW[ii] / d[ii]) + W[Pl] @ (TZ[ii] / d[ii]))
                beta = -fac.tval[a:b]
                UP = U_loc[P]
                betabar = -Tbar - UP @ epsbar
                G = UP @ UP.T / (N - 1) + lam * np.eye(P.size)
                s = sla.cho_solve(sla.cho_factor(G, lower=True), betabar)
                dlam -= float(s @ beta)
                u = U_loc[i]
                Ubar_loc[P] += (np.outer(s, u) - np.outer(s, beta @ UP) - np.outer(beta, s @ UP)) / (N - 1) \
                    - np.outer(beta, epsbar)
                Ubar_loc[i] += UP.T @ s / (N - 1)
        np.add.at(Ubar, pat.loc2glob, Ubar_loc)
    dXb += Ubar - Ubar.mean(axis=1, keepdims=True)
    return dXb, dlogR, dlam
