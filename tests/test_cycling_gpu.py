"""GPU parity of the assimilation cycle (Alg. 1) and of the RMSE of eq. (18).

- Perturbed observations drawn on the device (Philox4x64-10 + Box-Muller)
  against the oracle's draws, on a ragged member count (N = 21), on the
  96 x 48 grid (N = 40) and on the whole T-63 observation network
  (m = 26,726, N = 80), with seeds and cycle numbers beyond 32 bits.
- The squared error of the analysis mean (fp32 and fp64 ensembles, padded
  rows) against the oracle, and its bitwise repeatability.
- Sixteen cycles on the 96 x 48 grid (N = 40, r = 3, 8 x 4 sub-domains, 25%
  observed, zonal-shift forecast) against the oracle's cycle loop: squared
  error of every cycle, the RMSE, and the last analysis.
- Three cycles at the full T-63 size in bench.py's launch configuration: the
  third cycle's analysis on sampled sub-domains, recomputed by the oracle from
  the GPU's own background of that cycle, and its squared error.
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
from paper_1606_00807_amd.cycling import assimilate, rmse

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shift(geo, s):
    nl = int(sum(geo["nlev"]))

    def f(X):
        return torch.roll(X.reshape(nl, geo["ny"], geo["nx"], -1), s, dims=2).reshape(X.shape).contiguous()
    return f


@pytest.mark.parametrize("which,seed,cycle", [("small", 1, 0), ("small", 2**40 + 3, 2**35 + 1),
                                              ("grid", 2024, 7), ("t63", 5, 3)])
def test_perturbation_matches_oracle(which, seed, cycle):
    _need_gpu()
    if which == "small":
        p = synth.make_small(nx=12, ny=10, nlev=(3, 1), N=21, r_h=1, r_v=1, sdx=2, sdy=2, obs_frac=0.3,
                             ridge=1e-3, config=301)
    elif which == "grid":
        p = synth.make_grid2d()
    else:
        p = synth.make_t63()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    y = p.x_true[p.obs_idx]
    _say(f"[perturb {which}] m={p.m} N={p.N} seed={seed} cycle={cycle}")
    Ys = plan.perturb_observations(torch.as_tensor(y).cuda(), torch.as_tensor(p.r_diag).cuda(), seed, cycle)
    got = Ys.cpu().numpy()
    want = C.perturbed_observations(y, p.r_diag, seed, cycle, p.N)
    err = float(np.max(np.abs(got - want) / np.sqrt(p.r_diag)[:, None]))
    _say(f"[perturb {which}] max |dY| / sqrt(r) = {err:.2e}")
    assert got.shape == (p.m, p.N) and err <= 1e-13


@pytest.mark.parametrize("dtype,pad", [(torch.float64, 0), (torch.float32, 0), (torch.float64, 3)])
def test_sq_error_matches_oracle(dtype, pad):
    _need_gpu()
    p = synth.make_grid2d()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    g = np.random.default_rng(8)
    wide = torch.as_tensor(g.standard_normal((p.n, p.N + pad))).to(dtype).cuda()
    Xa = wide[:, :p.N]
    x_ref = g.standard_normal(p.n)
    e1 = plan.analysis_sq_error(Xa, torch.as_tensor(x_ref).cuda())
    e2 = plan.analysis_sq_error(Xa, torch.as_tensor(x_ref).cuda())
    want = C.sq_error(Xa.cpu().double().numpy(), x_ref)
    rel = abs(float(e1) - want) / want
    _say(f"[sq_error {dtype} pad={pad}] {float(e1):.12e} oracle {want:.12e} rel {rel:.1e}")
    assert rel <= 1e-12 and float(e1) == float(e2)


@pytest.mark.parametrize("mode,cycles", [("batched", 16), ("plain", 4)])
def test_cycles_match_oracle(mode, cycles):
    _need_gpu()
    p = synth.make_grid2d()
    obs = synth.cycle_truth_and_obs(p, cycles)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    r = torch.as_tensor(p.r_diag).cuda()
    out = assimilate(plan, torch.as_tensor(p.Xb).cuda(), [torch.as_tensor(y).cuda() for _, y in obs], r,
                     p.ridge, _shift(p.geometry, 1), seed=2024, x_ref=[torch.as_tensor(x).cuda() for x, _ in obs],
                     mode=mode)
    _say(f"[cycles {mode}] GPU rmse {out.rmse:.10e}")
    ora = C.assimilate(p.geometry, p.Xb, [y for _, y in obs], p.obs_idx, p.r_diag, p.ridge,
                       lambda X: synth.linear_forecast(X, p.geometry, 1), seed=2024, x_ref=[x for x, _ in obs])
    sq = out.sq_err.cpu().numpy()
    e_sq = float(np.max(np.abs(sq - ora.sq_err) / ora.sq_err))
    e_rmse = abs(out.rmse - ora.rmse) / ora.rmse
    xa = out.Xa.cpu().numpy().mean(1)
    xo = ora.Xa.mean(1)
    e_xa = float(np.linalg.norm(xa - xo) / np.linalg.norm(xo))
    _say(f"[cycles {mode}] oracle rmse {ora.rmse:.10e}; rel err sq_err {e_sq:.1e} rmse {e_rmse:.1e} "
         f"last X_a mean {e_xa:.1e}")
    # the filter must do its job: the first analysis is closer to the truth
    # than the background, and cycling lowers the error further
    e_b = float(np.linalg.norm(p.Xb.mean(1) - obs[0][0]) ** 2)
    assert sq[0] < 0.75 * e_b and float(np.mean(sq)) < 0.5 * e_b
    assert e_sq <= 1e-6 and e_rmse <= 1e-6 and e_xa <= 1e-6
    assert out.rmse == pytest.approx(rmse(sq), rel=1e-15)


def test_t63_cycles_sampled_subdomains_match_oracle():
    _need_gpu()
    p = synth.make_t63()
    obs = synth.cycle_truth_and_obs(p, 3)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    r = torch.as_tensor(p.r_diag).cuda()
    ys = [torch.as_tensor(y).cuda() for _, y in obs]
    refs = [torch.as_tensor(x).cuda() for x, _ in obs]
    fore = _shift(p.geometry, 1)
    _say(f"[t63 cycles] n={p.n} N={p.N} m={p.m}")
    first = assimilate(plan, torch.as_tensor(p.Xb).cuda(), ys[:2], r, p.ridge, fore, seed=11, x_ref=refs[:2])
    Xb2 = fore(first.Xa)
    last = assimilate(plan, Xb2, ys[2:], r, p.ridge, fore, seed=11, x_ref=refs[2:], first_cycle=2)
    _say(f"[t63 cycles] squared errors {first.sq_err.cpu().tolist()} {last.sq_err.cpu().tolist()}")
    Xa2 = last.Xa.cpu().numpy()
    want = C.sq_error(Xa2, obs[2][0])
    assert abs(float(last.sq_err[0]) - want) <= 1e-12 * want
    # the third cycle, recomputed by the oracle on sampled sub-domains from the GPU's own background
    X64 = Xb2.cpu().numpy().astype(np.float64)
    Ys = C.perturbed_observations(obs[2][1], p.r_diag, 11, 2, p.N)
    _, U = OF.anomalies(X64)
    for k in [6 * 24 + 11, 0, 287]:
        pat = OG.subdomain_pattern(p.geometry, k, p.obs_idx)
        fac = OF.fit_subdomain(U, pat, p.ridge)
        Z = A.solve_subdomain(fac, A.innovations(X64, Ys, p.obs_idx, pat), p.r_diag)
        rows = pat.loc2glob[pat.interior]
        ref = X64[rows] + Z[pat.interior]
        em = float(np.linalg.norm(Xa2[rows].mean(1) - ref.mean(1)) / np.linalg.norm(ref.mean(1)))
        ei = float(np.linalg.norm((Xa2[rows] - X64[rows]).mean(1) - Z[pat.interior].mean(1))
                   / np.linalg.norm(Z[pat.interior].mean(1)))
        _say(f"[t63 cycles] cycle 2 sub-domain {k}: X_a mean {em:.2e}, increment mean {ei:.2e}")
        assert em <= 1e-6 and ei <= 1e-5
