"""GPU parity on the uneven batch: 64 single-variable instances, grids from
32x16 to 192x96, 1-7 levels, N in [20, 120], r in [1, 5], 2-30% observed,
ridge 1e-3, 8 x 8-point sub-domains.

These instances reach sizes the T-63 workload does not: N up to 120 and up
to 181 predecessors (systems of 6-8 tiles in the one-wavefront fit and its
adjoint), and blocks with more than 128 observations (several observation
tiles per dual-form wavefront).  Every regression of every instance must run
on the one-wavefront kernels (none in the plain fallback bucket).

Every instance runs whole on the GPU.  The oracle recomputes one sampled
sub-domain per instance (T, D, local increments, X_a on its interior), and the
whole adjoint of four small instances.
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

PARAMS = synth.instance_params()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("k", range(len(PARAMS)))
def test_instance_sampled_subdomain_matches_oracle(k):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_instance(k, PARAMS)
    d = PARAMS[k]
    plan = Plan(p.geometry, p.N, p.obs_idx)
    _say(f"[instance {k}] {d['nx']}x{d['ny']}x{d['nlev']} N={p.N} r={d['r']} m={p.m} "
         f"max_p={plan.info['max_p']} max_block_obs={plan.info['max_block_obs']} "
         f"rows wave/plain={plan.info['fit_rows_wave']}/{plan.info['fit_rows_plain']}")
    assert plan.info["fit_rows_plain"] == 0 and plan.info["fit_rows_wave"] == plan.info["n_fit"]
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    Xa = plan.analyze(Xb, p.Y, p.r_diag).cpu().numpy()
    nsd = p.geometry["sdx"] * p.geometry["sdy"]
    ks = int(np.random.default_rng(1000 + k).integers(0, nsd))
    pat = OG.subdomain_pattern(p.geometry, ks, p.obs_idx)
    _, U = OF.anomalies(p.Xb)
    fac = OF.fit_subdomain(U, pat, p.ridge)
    X64 = np.asarray(p.Xb, np.float64)
    Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
    tval, dd = plan.factors(ks)
    et = _rel(tval, fac.tval) if fac.tval.size else 0.0
    ed = float(np.max(np.abs(dd - fac.d) / fac.d))
    ez = _rel(plan.increment(ks), Z) if np.any(Z) else 0.0
    rows = pat.loc2glob[pat.interior]
    ref = X64[rows] + Z[pat.interior]
    em = float(np.linalg.norm(Xa[rows].mean(1) - ref.mean(1)) / np.linalg.norm(ref.mean(1)))
    _say(f"[instance {k}] sub-domain {ks}: T={et:.2e} D={ed:.2e} Z={ez:.2e} X_a mean={em:.2e}")
    assert et <= 1e-9 and ed <= 1e-9 and ez <= 1e-8 and em <= 1e-6


# instances that cover N > 80 (up to 120: 8-tile kernel-form and p-form
# systems in instance 54), p > 128 and blocks with > 128 observations
@pytest.mark.parametrize("k", [1, 7, 20, 52, 54])
def test_instance_adjoint_matches_oracle(k):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_instance(k, PARAMS)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    _say(f"[instance {k} adjoint] n={p.n} N={p.N} m={p.m} max_p={plan.info['max_p']} "
         f"max_block_obs={plan.info['max_block_obs']}")
    assert plan.info["fit_rows_plain"] == 0
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    G = 2.0 * (res.Xa - p.x_true[:, None])
    dXb_o, dlogR_o, dlam_o = J.analyze_backward(p.Xb, p.obs_idx, p.r_diag, p.ridge, res, G)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    Xa = plan.analyze(Xb, p.Y, p.r_diag).cpu().numpy()
    dXb, dlogR, dlam = plan.backward(Xb, torch.as_tensor(G).cuda())
    ea = float(np.linalg.norm(Xa.mean(1) - res.Xa.mean(1)) / np.linalg.norm(res.Xa.mean(1)))
    e = [float(np.linalg.norm(dXb.cpu().numpy() - dXb_o) / np.linalg.norm(dXb_o)),
         float(np.linalg.norm(dlogR.cpu().numpy() - dlogR_o) / np.linalg.norm(dlogR_o)),
         abs(float(dlam) - dlam_o) / abs(dlam_o)]
    _say(f"[instance {k} adjoint] X_a mean {ea:.2e}; dX_b {e[0]:.2e} dlog r {e[1]:.2e} dlam {e[2]:.2e}")
    assert ea <= 1e-6 and max(e) <= 1e-5
