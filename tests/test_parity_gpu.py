"""GPU parity: the HIP path against the FP64 oracle on identical seeded inputs.

Tolerances (relative to the largest magnitude of each quantity):
  T values, D        1e-9   (FP64 both sides; only the summation order differs,
                             amplified by cond(G) <= ~1e5 of the regressions)
  local increments   1e-8
  analysis mean      1e-6   (the acceptance gate; reported values are far smaller)
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import analysis as A
from paper_1606_00807_amd import EnkfmcError, Plan

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "ring40": lambda: synth.make_ring(),
    "multivar_3d": lambda: synth.make_small(nx=12, ny=10, nlev=(3, 1), N=20, r_h=1, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.3, config=201),
    "kernel_form": lambda: synth.make_small(nx=12, ny=10, nlev=(3,), N=8, r_h=1, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.3, ridge=1e-2, config=202),
    "mixed_forms": lambda: synth.make_small(nx=14, ny=12, nlev=(3,), N=24, r_h=2, r_v=1, sdx=2, sdy=2,
                                            obs_frac=0.25, ridge=1e-3, config=203),
    "nonperiodic_uneven": lambda: synth.make_small(nx=13, ny=11, nlev=(2, 1), N=20, r_h=2, r_v=1, sdx=3, sdy=2,
                                                   periodic_x=False, obs_frac=0.2, ridge=1e-3, config=204),
    "fp32_storage": lambda: synth.make_small(nx=12, ny=10, nlev=(3,), N=24, r_h=1, r_v=1, sdx=2, sdy=2,
                                             obs_frac=0.3, ridge=1e-3, config=205, dtype=np.float32),
    "grid96x48": lambda: synth.make_grid2d(),
    # p-form systems of 6-8 tiles (p up to 121 < N = 125)
    "pform_8tiles": lambda: synth.make_small(nx=16, ny=10, nlev=(3,), N=125, r_h=4, r_v=1, sdx=2, sdy=2,
                                             obs_frac=0.2, ridge=1e-3, config=208),
    # kernel-form systems of 8 tiles (N = 120, p up to 181)
    "kform_8tiles": lambda: synth.make_small(nx=20, ny=12, nlev=(3,), N=120, r_h=5, r_v=1, sdx=2, sdy=2,
                                             obs_frac=0.2, ridge=1e-3, config=209),
    # rows with more than 192 predecessors (r_h = 4, r_v = 2: up to 202) go to
    # the plain kernel, the others to the one-wavefront kernels
    "plain_bucket_p": lambda: synth.make_small(nx=12, ny=12, nlev=(5,), N=40, r_h=4, r_v=2, sdx=1, sdy=1,
                                               obs_frac=0.2, ridge=1e-2, config=210),
    # N > 128: every row with predecessors goes to the plain kernel
    "plain_bucket_N": lambda: synth.make_small(nx=10, ny=8, nlev=(2,), N=136, r_h=1, r_v=1, sdx=2, sdy=2,
                                               obs_frac=0.3, ridge=1e-3, config=211),
}

# expected split of the batched fit between the one-wavefront kernels and
# the plain fallback bucket
SPLIT = {"plain_bucket_p": "both", "plain_bucket_N": "both"}


def _rel(a, b):
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def _run(p, mode):
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge, mode=mode)
    Xa = plan.analyze(Xb, p.Y, p.r_diag)
    torch.cuda.synchronize()
    return plan, Xa.cpu().numpy()


@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("case", list(CASES))
def test_fit_and_analysis_match_oracle(case, mode):
    _need_gpu()
    p = CASES[case]()
    _say(f"[parity] case={case} mode={mode} n={p.n} N={p.N} m={p.m}")
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    plan, Xa = _run(p, mode)
    worst_t = worst_d = worst_z = 0.0
    for k, (fac, Z) in enumerate(zip(res.factors, res.Z)):
        tval, d = plan.factors(k)
        if fac.tval.size:
            worst_t = max(worst_t, _rel(tval, fac.tval))
        worst_d = max(worst_d, float(np.max(np.abs(d - fac.d) / fac.d)))
        if np.any(Z):
            worst_z = max(worst_z, _rel(plan.increment(k), Z))
    info = plan.info
    if case in SPLIT:
        assert info["fit_rows_plain"] > 0 and info["fit_rows_wave"] > 0, info
    else:
        assert info["fit_rows_plain"] == 0 and info["fit_rows_wave"] == info["n_fit"], info
    if mode == "batched":   # the timing of the last fit names the kernels that ran
        plan.set_timing(True)
        plan.fit(torch.as_tensor(p.Xb).cuda(), p.ridge, mode=mode)
        ph = plan.timing()
        plan.set_timing(False)
        assert (ph["fit_fallback"] > 0) == (case in SPLIT), ph
    mean_rel = float(np.linalg.norm(Xa.mean(1) - res.Xa.mean(1)) / np.linalg.norm(res.Xa.mean(1)))
    inc_rel = float(np.linalg.norm((Xa - res.Xa)) / max(np.linalg.norm(res.Xa - p.Xb), 1e-300))
    _say(f"[parity] case={case} mode={mode} T={worst_t:.2e} D={worst_d:.2e} Z={worst_z:.2e} "
         f"mean={mean_rel:.2e} increment={inc_rel:.2e}")
    assert worst_t <= 1e-9
    assert worst_d <= 1e-9
    assert worst_z <= 1e-8
    assert mean_rel <= 1e-6
    assert inc_rel <= 1e-8


def test_no_observations_leaves_background_bitwise():
    _need_gpu()
    p = synth.make_small(nx=10, ny=8, nlev=(2,), N=16, r_h=1, r_v=1, sdx=2, sdy=2, obs_frac=0.0, config=206)
    plan, Xa = _run(p, "batched")
    assert np.array_equal(Xa, p.Xb)


def test_fit_reports_singular_regression():
    """lam = 0 with p >= N - 1: the device reports ENOTSPD (forced from the host by the input sizes)."""
    _need_gpu()
    p = synth.make_small(nx=9, ny=7, nlev=(3,), N=6, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=0.2, config=207)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    for mode in ("plain", "batched"):
        with pytest.raises(EnkfmcError) as e:
            plan.fit(torch.as_tensor(p.Xb).cuda(), 0.0, mode=mode)
        assert e.value.code == "ENOTSPD"


def test_analyze_before_fit_is_a_state_error():
    _need_gpu()
    p = synth.make_ring()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    plan.ensure_workspace()
    with pytest.raises(EnkfmcError) as e:
        plan.analyze(torch.as_tensor(p.Xb).cuda(), p.Y, p.r_diag)
    assert e.value.code == "ESTATE"
