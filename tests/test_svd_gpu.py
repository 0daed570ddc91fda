"""GPU parity of the SVD fit (ENKFMC_FIT_SVD, the route of Section 5) against
the oracle's SVD regression (oracle.fit.fit_row_svd, itself pinned against
the normal equations, lstsq and closed forms in test_oracle_pins.py).

Same tolerances as the Cholesky fit: T, D within 1e-9 of the largest entry,
local increments 1e-8, analysis mean 1e-6.  Also at the full T-63 size on
sampled sub-domains, and the SVD mode's coefficients against the batched
Cholesky fit of the same plan over the whole state.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import analysis as A
from oracle import fit as OF
from oracle import geometry as OG
from paper_1606_00807_amd import EnkfmcError, Plan

pytestmark = pytest.mark.gpu

CASES = {
    "ring40": lambda: synth.make_ring(),
    "multivar_3d": lambda: synth.make_small(nx=12, ny=10, nlev=(3, 1), N=20, r_h=1, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.3, config=201),
    "kernel_form": lambda: synth.make_small(nx=12, ny=10, nlev=(3,), N=8, r_h=1, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.3, ridge=1e-2, config=202),
    "mixed_forms": lambda: synth.make_small(nx=14, ny=12, nlev=(3,), N=24, r_h=2, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.25, ridge=1e-3, config=203),
    "fp32_storage": lambda: synth.make_small(nx=12, ny=10, nlev=(3,), N=24, r_h=1, r_v=1, sdx=2, sdy=2,
                                             obs_frac=0.3, ridge=1e-3, config=205, dtype=np.float32),
    "grid96x48": lambda: synth.make_grid2d(),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _svd_factors(p, pat):
    _, U = OF.anomalies(p.Xb)
    return OF.fit_subdomain(U, pat, p.ridge, method="svd")


@pytest.mark.parametrize("case", list(CASES))
def test_svd_fit_and_analysis_match_oracle(case):
    p = CASES[case]()
    _say(f"[svd] case={case} n={p.n} N={p.N} m={p.m} ridge={p.ridge}")
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="svd")
    Xa = plan.analyze(Xb, p.Y, p.r_diag).cpu().numpy()
    X64 = np.asarray(p.Xb, np.float64)
    nsd = p.geometry["sdx"] * p.geometry["sdy"]
    ks = range(nsd) if nsd <= 8 else [0, nsd // 2 + 1, nsd - 1]
    worst_t = worst_d = worst_z = 0.0
    diff2 = ref2 = 0.0
    for k in ks:
        pat = OG.subdomain_pattern(p.geometry, k, p.obs_idx)
        fac = _svd_factors(p, pat)
        Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
        tval, d = plan.factors(k)
        if fac.tval.size:
            worst_t = max(worst_t, _rel(tval, fac.tval))
        worst_d = max(worst_d, float(np.max(np.abs(d - fac.d) / fac.d)))
        if np.any(Z):
            worst_z = max(worst_z, _rel(plan.increment(k), Z))
        rows = pat.loc2glob[pat.interior]
        ref = X64[rows] + Z[pat.interior]
        diff2 += float(np.sum((Xa[rows].mean(1) - ref.mean(1)) ** 2))
        ref2 += float(np.sum(ref.mean(1) ** 2))
    mean_rel = float(np.sqrt(diff2 / ref2))
    _say(f"[svd] case={case} T={worst_t:.2e} D={worst_d:.2e} Z={worst_z:.2e} mean={mean_rel:.2e}")
    assert worst_t <= 1e-9 and worst_d <= 1e-9 and worst_z <= 1e-8 and mean_rel <= 1e-6


def test_svd_without_ridge_reports_singular_regression():
    """lam = 0 with p >= N - 1 is ENOTSPD in the SVD mode as well (no pseudo-inverse)."""
    p = synth.make_small(nx=9, ny=7, nlev=(3,), N=6, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.2, config=207)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    with pytest.raises(EnkfmcError) as e:
        plan.fit(torch.as_tensor(p.Xb).cuda(), 0.0, mode="svd")
    assert e.value.code == "ENOTSPD"


@pytest.fixture(scope="module")
def t63_svd():
    p = synth.make_t63()
    _say(f"[svd t63] n={p.n} N={p.N} m={p.m}")
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    chol = [plan.factors(k) for k in (0, 6 * 24 + 11, 287)]
    plan.fit(Xb, p.ridge, mode="svd")
    Xa = plan.analyze(Xb, p.Y, p.r_diag)
    torch.cuda.synchronize()
    return p, plan, Xa.cpu().numpy(), chol


@pytest.mark.parametrize("k", [6 * 24 + 11, 0])
def test_svd_t63_sampled_subdomain_matches_oracle(t63_svd, k):
    p, plan, Xa, _ = t63_svd
    pat = OG.subdomain_pattern(p.geometry, k, p.obs_idx)
    fac = _svd_factors(p, pat)
    X64 = np.asarray(p.Xb, np.float64)
    Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
    tval, d = plan.factors(k)
    et, ed = _rel(tval, fac.tval), float(np.max(np.abs(d - fac.d) / fac.d))
    ez = _rel(plan.increment(k), Z)
    rows = pat.loc2glob[pat.interior]
    ref = X64[rows] + Z[pat.interior]
    em = float(np.linalg.norm(Xa[rows].mean(1) - ref.mean(1)) / np.linalg.norm(ref.mean(1)))
    _say(f"[svd t63] sub-domain {k}: T={et:.2e} D={ed:.2e} Z={ez:.2e} X_a mean={em:.2e}")
    assert et <= 1e-9 and ed <= 1e-9 and ez <= 1e-8 and em <= 1e-6


def test_svd_t63_matches_cholesky_fit(t63_svd):
    """The two routes give the same coefficients (eq. 1): SVD against the
    batched Cholesky fit of the same plan on three whole sub-domains."""
    p, plan, _, chol = t63_svd
    for k, (tc, dc) in zip((0, 6 * 24 + 11, 287), chol):
        ts, ds = plan.factors(k)
        et, ed = _rel(ts, tc), float(np.max(np.abs(ds - dc) / dc))
        _say(f"[svd t63] sub-domain {k}: SVD vs Cholesky T={et:.2e} D={ed:.2e}")
        assert et <= 1e-9 and ed <= 1e-9
