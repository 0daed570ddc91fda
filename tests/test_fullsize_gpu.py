"""GPU checks at the full T-63 size (192x96, 7 levels x {u, v, T, q} + ps,
n = 534,528, N = 80, r_h = 4, r_v = 1, 24 x 12 sub-domains, 5% observed,
ridge 1e-3), in the launch configuration bench.py times.

The oracle cannot redo the whole state quickly, so it recomputes samples:
  - T, D, local increments and X_a of sampled sub-domains (a mid-latitude
    one, the first one and one clipped at the pole);
  - the adjoint on a 4 x 4-point patch at a sub-domain corner: the patch
    lies in the extended boxes of exactly four sub-domains, so the oracle's
    adjoint restricted to those four gives dX_b and dlog r there exactly;
and directional finite differences of L = <Gbar, X_a> (Richardson-extrapolated
central differences, eight random directions for X_b and for log r, and the
ridge) check the GPU adjoint against the GPU forward pass over the whole state.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as J
from oracle import analysis as A
from oracle import fit as OF
from oracle import geometry as OG
from paper_1606_00807_amd import Plan

pytestmark = pytest.mark.gpu

SDX = 24


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def t63():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_t63()
    _say(f"[t63] n={p.n} N={p.N} m={p.m}")
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    Xa = plan.analyze(Xb, p.Y, p.r_diag)
    torch.cuda.synchronize()
    return p, plan, Xb, Xa


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("k", [6 * SDX + 11, 0, 3])
def test_t63_sampled_subdomain_matches_oracle(t63, k):
    p, plan, Xb, Xa = t63
    pat = OG.subdomain_pattern(p.geometry, k, p.obs_idx)
    mean, U = OF.anomalies(p.Xb)
    fac = OF.fit_subdomain(U, pat, p.ridge)
    X64 = np.asarray(p.Xb, np.float64)
    Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
    tval, d = plan.factors(k)
    rows = pat.loc2glob[pat.interior]
    xa = Xa[torch.as_tensor(rows).cuda()].cpu().numpy()
    xa_ref = X64[rows] + Z[pat.interior]
    et, ed = _rel(tval, fac.tval), float(np.max(np.abs(d - fac.d) / fac.d))
    ez = _rel(plan.increment(k), Z)
    em = float(np.linalg.norm(xa.mean(1) - xa_ref.mean(1)) / np.linalg.norm(xa_ref.mean(1)))
    _say(f"[t63] sub-domain {k}: n_sd={pat.n_sd} T={et:.2e} D={ed:.2e} Z={ez:.2e} X_a mean={em:.2e}")
    assert et <= 1e-9 and ed <= 1e-9 and ez <= 1e-8 and em <= 1e-6


def _patch(p, lon0, lat0, size=4):
    nx, ny = p.geometry["nx"], p.geometry["ny"]
    out = []
    off = 0
    for L in p.geometry["nlev"]:
        for lev in range(L):
            for lat in range(lat0, lat0 + size):
                for lon in range(lon0, lon0 + size):
                    out.append(off + (lev * ny + lat) * nx + lon)
        off += L * nx * ny
    return np.array(out)


def test_t63_adjoint_on_a_corner_patch_matches_oracle(t63):
    p, plan, Xb, Xa = t63
    g = np.random.default_rng(7)
    G = g.standard_normal((p.n, p.N))
    dXb, dlogR, _ = plan.backward(Xb, torch.as_tensor(G).cuda())
    dXb = dXb.cpu().numpy()
    dlogR = dlogR.cpu().numpy()
    # tiles are 8 x 8 with a halo of 4: lon 88..91 x lat 48..51 lies in the
    # boxes of tiles (10|11, 5|6) and of no other
    ks = [5 * SDX + 10, 5 * SDX + 11, 6 * SDX + 10, 6 * SDX + 11]
    rows = _patch(p, 88, 48)
    pats = [OG.subdomain_pattern(p.geometry, k, p.obs_idx) for k in ks]
    for k in range(p.geometry["sdx"] * p.geometry["sdy"]):
        if k in ks:
            continue
        kx, ky = k % SDX, k // SDX
        if abs(kx - 10.5) < 2 and abs(ky - 5.5) < 2:   # neighbours must not hold the patch
            assert not np.isin(rows, OG.subdomain_pattern(p.geometry, k, p.obs_idx).loc2glob).any()
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge, patterns=pats)
    _say("[t63] oracle adjoint on 4 sub-domains")
    dXb_o, dlogR_o, _ = J.analyze_backward(p.Xb, p.obs_idx, p.r_diag, p.ridge, res, G)
    e_x = float(np.linalg.norm(dXb[rows] - dXb_o[rows]) / np.linalg.norm(dXb_o[rows]))
    obs = np.nonzero(np.isin(p.obs_idx, rows))[0]
    assert obs.size > 5
    e_r = float(np.linalg.norm(dlogR[obs] - dlogR_o[obs]) / np.linalg.norm(dlogR_o[obs]))
    _say(f"[t63] patch of {rows.size} components, {obs.size} observed: dX_b rel {e_x:.2e}, dlog r rel {e_r:.2e}")
    assert e_x <= 1e-5 and e_r <= 1e-5


def test_t63_adjoint_directional_finite_differences(t63):
    """fp64 storage of the same state so that the perturbations are exact."""
    p, plan, _, _ = t63
    X = torch.as_tensor(np.asarray(p.Xb, np.float64)).cuda()
    Y = torch.as_tensor(p.Y).cuda()
    r0 = torch.as_tensor(p.r_diag).cuda()
    g = np.random.default_rng(9)
    G = torch.as_tensor(g.standard_normal((p.n, p.N))).cuda()

    def L(Xb, r, lam):
        plan.fit(Xb, lam)
        return float(torch.sum(G * plan.analyze(Xb, Y, r)))

    L(X, r0, p.ridge)
    dXb, dlogR, dlam = plan.backward(X, G)

    def richardson(f, h):
        # central differences at h and h/2 combined to cancel the h^2 term
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    for d in range(8):   # eight random directions per parameter group
        V = torch.as_tensor(g.standard_normal((p.n, p.N))).cuda()
        fd = richardson(lambda e: L(X + e * V, r0, p.ridge), 1e-4)
        ad = float(torch.sum(dXb * V))
        _say(f"[t63 fd {d}] X_b: fd={fd:.10e} adjoint={ad:.10e}")
        assert abs(fd - ad) <= 1e-6 * abs(fd)
        v = torch.as_tensor(g.standard_normal(p.m)).cuda()
        fd = richardson(lambda e: L(X, r0 * torch.exp(e * v), p.ridge), 1e-4)
        ad = float(torch.sum(dlogR * v))
        _say(f"[t63 fd {d}] log r: fd={fd:.10e} adjoint={ad:.10e}")
        assert abs(fd - ad) <= 1e-6 * abs(fd)
    fd = richardson(lambda e: L(X, r0, p.ridge + e), 1e-6)
    _say(f"[t63 fd] lam: fd={fd:.10e} adjoint={float(dlam):.10e}")
    assert abs(fd - float(dlam)) <= 1e-6 * abs(fd)


def test_t63_adjoint_with_factor_cache_matches_recompute(t63):
    """The reverse pass from the kernel-form factors cached by the fit (about
    33 GB at T-63) against the one that recomputes each row's Gram and
    Cholesky: equal up to rounding (the cached path forms L^-1 v by forward
    substitution instead of inside the elimination)."""
    p, plan, Xb, _ = t63
    G = torch.as_tensor(np.random.default_rng(11).standard_normal((p.n, p.N))).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    plan.analyze(Xb, p.Y, p.r_diag)
    ref = [t.cpu().numpy() for t in plan.backward(Xb, G)]
    nbytes = plan.set_factor_cache(True)
    try:
        _say(f"[t63] factor cache {nbytes / 2**30:.2f} GiB")
        assert nbytes == plan.info["factor_cache_bytes"] > 0
        plan.fit(Xb, p.ridge, mode="batched")
        plan.analyze(Xb, p.Y, p.r_diag)
        got = [t.cpu().numpy() for t in plan.backward(Xb, G)]
        errs = [float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))) for a, b in zip(got, ref)]
        _say(f"[t63] cached vs recomputed: dX_b {errs[0]:.2e}, dlog r {errs[1]:.2e}, dlam {errs[2]:.2e}")
        assert max(errs) <= 1e-9
    finally:
        plan.set_factor_cache(False)
