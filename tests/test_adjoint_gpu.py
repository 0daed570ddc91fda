"""GPU parity of the adjoint (enkfmc_analyze_backward) against the FP64 oracle.

Tolerance: 2-norm relative error <= 1e-5 for each of dX_b, dlog r and dlam
(both sides FP64; the adjoint re-solves the same systems, so the error is of
the order of cond(A) * 1e-16).  Also checked: bitwise repeatability, central
finite differences of the GPU forward pass, and the torch.autograd wrapper.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as J
from oracle import analysis as A
from paper_1606_00807_amd import Plan, enkfmc_analysis

pytestmark = pytest.mark.gpu

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
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _gpu_forward(p, plan, Xb, mode="batched"):
    plan.fit(Xb, p.ridge, mode=mode)
    return plan.analyze(Xb, p.Y, p.r_diag)


@pytest.mark.parametrize("mode", ["plain", "batched"])
@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_matches_oracle(case, mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = CASES[case]()
    _say(f"[adjoint] {case} mode={mode} n={p.n} N={p.N} m={p.m} ridge={p.ridge}")
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    Gbar = 2.0 * (res.Xa - p.x_true[:, None])
    dXb_o, dlogR_o, dlam_o = J.analyze_backward(p.Xb, p.obs_idx, p.r_diag, p.ridge, res, Gbar)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    _gpu_forward(p, plan, Xb, mode)
    dXb, dlogR, dlam = plan.backward(Xb, torch.as_tensor(Gbar).cuda())
    torch.cuda.synchronize()
    e = (_rel2(dXb.cpu().numpy(), dXb_o), _rel2(dlogR.cpu().numpy(), dlogR_o),
         abs(float(dlam) - dlam_o) / max(abs(dlam_o), 1e-300) if p.ridge > 0 else abs(float(dlam) - dlam_o))
    _say(f"[adjoint] {case} rel err dXb={e[0]:.2e} dlogR={e[1]:.2e} dlam={e[2]:.2e} (dlam={float(dlam):.6e})")
    assert e[0] <= 1e-5 and e[1] <= 1e-5 and e[2] <= 1e-5


@pytest.mark.parametrize("case", ["kernel_form", "mixed_forms", "nonperiodic_uneven"])
def test_factor_cache_adjoint_matches_recompute_and_oracle(case):
    """enkfmc_plan_set_factor_cache: the batched fit keeps the kernel-form
    rows' Cholesky tiles and the reverse pass reads them.  Equal to the
    recomputing reverse pass up to rounding (1e-9), to the oracle within the
    adjoint tolerance, bitwise repeatable; dropping the cache brings back the
    recomputing pass bit for bit."""
    p = CASES[case]()
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    Gbar = 2.0 * (res.Xa - p.x_true[:, None])
    dXb_o, dlogR_o, dlam_o = J.analyze_backward(p.Xb, p.obs_idx, p.r_diag, p.ridge, res, Gbar)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    G = torch.as_tensor(Gbar).cuda()
    _gpu_forward(p, plan, Xb)
    ref = [t.cpu().numpy() for t in plan.backward(Xb, G)]
    nbytes = plan.set_factor_cache(True)
    _say(f"[cache] {case} n={p.n} N={p.N} cache {nbytes} bytes")
    assert nbytes == plan.info["factor_cache_bytes"] > 0
    _gpu_forward(p, plan, Xb)
    got = [t.cpu().numpy() for t in plan.backward(Xb, G)]
    again = [t.cpu().numpy() for t in plan.backward(Xb, G)]
    e_ref = [_rel2(a, b) for a, b in zip(got, ref)]
    e_or = [_rel2(got[0], dXb_o), _rel2(got[1], dlogR_o), abs(float(got[2]) - dlam_o) / abs(dlam_o)]
    _say(f"[cache] {case} vs recompute {e_ref[0]:.2e} {e_ref[1]:.2e} {e_ref[2]:.2e}; "
         f"vs oracle {e_or[0]:.2e} {e_or[1]:.2e} {e_or[2]:.2e}")
    assert max(e_ref) <= 1e-9 and max(e_or) <= 1e-5
    assert all(np.array_equal(a, b) for a, b in zip(got, again))
    assert plan.set_factor_cache(False) == 0
    _gpu_forward(p, plan, Xb)
    back = [t.cpu().numpy() for t in plan.backward(Xb, G)]
    assert all(np.array_equal(a, b) for a, b in zip(back, ref))


def test_adjoint_is_bitwise_repeatable():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = CASES["mixed_forms"]()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    _gpu_forward(p, plan, Xb)
    G = torch.as_tensor(np.random.default_rng(5).standard_normal((p.n, p.N))).cuda()
    a = [t.clone() for t in plan.backward(Xb, G)[:2]] + [plan.backward(Xb, G)[2].clone()]
    b = plan.backward(Xb, G)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


def test_adjoint_matches_finite_differences_of_gpu_forward():
    """Central differences of L = ||X_a - x_true 1^T||^2 computed on the GPU."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_small(nx=10, ny=8, nlev=(2,), N=12, r_h=1, r_v=1, sdx=2, sdy=2, obs_frac=0.3, ridge=0.05,
                         config=111)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    xt = torch.as_tensor(p.x_true).cuda()[:, None]

    def loss(Xb_np, r, lam):
        Xb = torch.as_tensor(Xb_np).cuda()
        plan.fit(Xb, lam)
        Xa = plan.analyze(Xb, p.Y, r)
        return float(torch.sum((Xa - xt) ** 2)), Xb, Xa

    L0, Xb, Xa = loss(p.Xb, p.r_diag, p.ridge)
    dXb, dlogR, dlam = plan.backward(Xb, 2.0 * (Xa - xt))
    dXb, dlogR, dlam = dXb.cpu().numpy(), dlogR.cpu().numpy(), float(dlam)
    g = np.random.default_rng(11)
    h = 1e-5
    V = g.standard_normal(p.Xb.shape)
    fd = (loss(p.Xb + h * V, p.r_diag, p.ridge)[0] - loss(p.Xb - h * V, p.r_diag, p.ridge)[0]) / (2 * h)
    _say(f"[fd] X_b: fd={fd:.10e} adjoint={np.sum(dXb * V):.10e}")
    assert abs(fd - np.sum(dXb * V)) <= 1e-6 * max(1.0, abs(fd))
    v = g.standard_normal(p.m)
    lr = np.log(p.r_diag)
    fd = (loss(p.Xb, np.exp(lr + h * v), p.ridge)[0] - loss(p.Xb, np.exp(lr - h * v), p.ridge)[0]) / (2 * h)
    _say(f"[fd] log r: fd={fd:.10e} adjoint={dlogR @ v:.10e}")
    assert abs(fd - dlogR @ v) <= 1e-6 * max(1.0, abs(fd))
    fd = (loss(p.Xb, p.r_diag, p.ridge + h)[0] - loss(p.Xb, p.r_diag, p.ridge - h)[0]) / (2 * h)
    _say(f"[fd] lam: fd={fd:.10e} adjoint={dlam:.10e}")
    assert abs(fd - dlam) <= 1e-6 * max(1.0, abs(fd))


def test_autograd_function_matches_direct_backward():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = CASES["mixed_forms"]()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda().requires_grad_(True)
    logr = torch.log(torch.as_tensor(p.r_diag)).cuda().requires_grad_(True)
    lam = torch.tensor(p.ridge, dtype=torch.float64, device="cuda", requires_grad=True)
    Y = torch.as_tensor(p.Y).cuda()
    Xa = enkfmc_analysis(Xb, logr, lam, plan, Y)
    loss = torch.sum((Xa - torch.as_tensor(p.x_true).cuda()[:, None]) ** 2)
    loss.backward()
    dXb, dlogR, dlam = plan.backward(Xb.detach(), 2.0 * (Xa.detach() - torch.as_tensor(p.x_true).cuda()[:, None]))
    assert torch.equal(Xb.grad, dXb) and torch.equal(logr.grad, dlogR) and torch.equal(lam.grad, dlam.reshape(()))


def test_autograd_refuses_observations_overwritten_in_place():
    """The reverse pass reads the Y of its forward call: refilling that
    tensor in place before backward() must raise, not give gradients of
    another analysis."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = CASES["mixed_forms"]()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda().requires_grad_(True)
    logr = torch.log(torch.as_tensor(p.r_diag)).cuda().requires_grad_(True)
    Y = torch.as_tensor(p.Y).cuda()
    Xa = enkfmc_analysis(Xb, logr, p.ridge, plan, Y)
    loss = torch.sum(Xa ** 2)
    Y.add_(1.0)   # e.g. the next cycle's perturbed observations drawn into the same buffer
    with pytest.raises(RuntimeError, match="modified by an inplace operation"):
        loss.backward()


def test_backward_without_analysis_is_a_state_error():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_00807_amd import EnkfmcError
    p = CASES["ring40"]()
    plan = Plan(p.geometry, p.N, p.obs_idx)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge)
    with pytest.raises(EnkfmcError):
        plan.backward(Xb, torch.zeros_like(Xb))
