"""Accuracy against the number of sub-domains at a fixed radius (the synthetic
analogue of the paper's Section 4.3, which reports nearly the same RMSE for
every processor count).

96 x 48 grid, N = 40, r = 3, 25% observed, ridge 0, zonal-shift forecast,
sub-domains Delta = 2x1, 4x2, 8x4, 16x8 (interiors 48x48 down to 6x6, halo 3):
  - every Delta: the GPU cycles equal the oracle's cycle loop (squared error
    of each cycle and the last analysis mean to 1e-6);
  - over eight cycles the RMSE of eq. (18) stays within 10% across Delta.
At the full T-63 size (N = 80, r_h = 4, r_v = 1) the analysis of sampled
sub-domains matches the oracle for Delta = 6x3 and 48x24 too (the blocks of
bench.py's sub-domain study).
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import analysis as A
from oracle import cycling as C
from oracle import fit as OF
from oracle import geometry as OG
from paper_1606_00807_amd import Plan
from paper_1606_00807_amd.cycling import assimilate

pytestmark = pytest.mark.gpu

DELTAS = [(2, 1), (4, 2), (8, 4), (16, 8)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _shift(geo):
    nl = int(sum(geo["nlev"]))

    def f(X):
        return torch.roll(X.reshape(nl, geo["ny"], geo["nx"], -1), 1, dims=2).reshape(X.shape).contiguous()
    return f


def _with_delta(p, sdx, sdy):
    geo = dict(p.geometry)
    geo["sdx"], geo["sdy"] = sdx, sdy
    return geo


def _gpu_cycles(p, geo, obs):
    plan = Plan(geo, p.N, p.obs_idx)
    return assimilate(plan, torch.as_tensor(p.Xb).cuda(), [torch.as_tensor(y).cuda() for _, y in obs],
                      torch.as_tensor(p.r_diag).cuda(), p.ridge, _shift(geo), seed=99,
                      x_ref=[torch.as_tensor(x).cuda() for x, _ in obs])


@pytest.mark.parametrize("sdx,sdy", DELTAS)
def test_cycles_match_oracle_for_every_delta(sdx, sdy):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_grid2d()
    geo = _with_delta(p, sdx, sdy)
    obs = synth.cycle_truth_and_obs(p, 3)
    out = _gpu_cycles(p, geo, obs)
    ora = C.assimilate(geo, p.Xb, [y for _, y in obs], p.obs_idx, p.r_diag, p.ridge,
                       lambda X: synth.linear_forecast(X, geo, 1), seed=99, x_ref=[x for x, _ in obs])
    sq = out.sq_err.cpu().numpy()
    e_sq = float(np.max(np.abs(sq - ora.sq_err) / ora.sq_err))
    xa, xo = out.Xa.cpu().numpy().mean(1), ora.Xa.mean(1)
    e_xa = float(np.linalg.norm(xa - xo) / np.linalg.norm(xo))
    _say(f"[delta {sdx}x{sdy}] sq_err {np.round(sq, 3).tolist()} rel err {e_sq:.1e}, last X_a mean {e_xa:.1e}")
    assert e_sq <= 1e-6 and e_xa <= 1e-6


def test_rmse_nearly_invariant_across_delta():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_grid2d()
    obs = synth.cycle_truth_and_obs(p, 8)
    rm = {}
    for sdx, sdy in DELTAS:
        rm[(sdx, sdy)] = _gpu_cycles(p, _with_delta(p, sdx, sdy), obs).rmse
    _say("[delta study] RMSE over 8 cycles: " + ", ".join(f"{a}x{b}: {v:.4f}" for (a, b), v in rm.items()))
    v = np.array(list(rm.values()))
    assert (v.max() - v.min()) / v.min() <= 0.10


@pytest.mark.parametrize("sdx,sdy,ks", [(6, 3, [0, 7, 17]), (48, 24, [0, 12 * 48 + 23, 1151])])
def test_t63_other_delta_sampled_subdomains_match_oracle(sdx, sdy, ks):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_t63()
    geo = _with_delta(p, sdx, sdy)
    plan = Plan(geo, p.N, p.obs_idx)
    _say(f"[t63 delta {sdx}x{sdy}] n_fit={plan.info['n_fit']} max_block_rows={plan.info['max_block_rows']} "
         f"max_block_obs={plan.info['max_block_obs']}")
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode="batched")
    Xa = plan.analyze(Xb, p.Y, p.r_diag).cpu().numpy()
    X64 = np.asarray(p.Xb, np.float64)
    _, U = OF.anomalies(X64)
    for k in ks:
        pat = OG.subdomain_pattern(geo, k, p.obs_idx)
        fac = OF.fit_subdomain(U, pat, p.ridge)
        Z = A.solve_subdomain(fac, A.innovations(X64, p.Y, p.obs_idx, pat), p.r_diag)
        rows = pat.loc2glob[pat.interior]
        ref = X64[rows] + Z[pat.interior]
        em = float(np.linalg.norm(Xa[rows].mean(1) - ref.mean(1)) / np.linalg.norm(ref.mean(1)))
        ez = float(np.max(np.abs(plan.increment(k) - Z)) / np.max(np.abs(Z)))
        _say(f"[t63 delta {sdx}x{sdy}] sub-domain {k}: n_sd={pat.n_sd} Z={ez:.2e} X_a mean={em:.2e}")
        assert em <= 1e-6 and ez <= 1e-8
