"""Sixteen assimilation cycles and the gradient through all of them.

Workload: the 96 x 48 grid (N = 40, r = 3, 8 x 4 sub-domains, 25% observed at
fixed sites, R = 0.05), ridge 1e-3.  Between cycles the synthetic forecast
shifts every field one cell eastward (exact and linear; its adjoint shifts
back); each cycle observes its own truth with fresh noise.  Loss
L = sum over cycles of ||X_a - x_true 1^T||^2, differentiated with respect to
the first background X_b, log diag(R) (shared by the cycles) and the ridge.

The GPU chain runs through the torch.autograd wrapper, which recomputes each
cycle's fit and analysis in the reverse pass.  It is compared with the oracle's
analytic gradient (the same chain rule over the oracle's per-cycle adjoint) to
1e-5, and with Richardson-extrapolated central differences of the GPU forward
chain along eight random directions for X_b and for log r, and the ridge.
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

CYCLES = 16


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _shift(X, geo, s):
    nl = int(sum(geo["nlev"]))
    return torch.roll(X.reshape(nl, geo["ny"], geo["nx"], -1), s, dims=2).reshape(X.shape)


@pytest.fixture(scope="module")
def chain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_grid2d(ridge=1e-3)
    obs = synth.cycle_observations(p, CYCLES)
    plan = Plan(p.geometry, p.N, p.obs_idx)
    truths = [torch.as_tensor(x).cuda()[:, None] for x, _ in obs]
    Ys = [torch.as_tensor(Y).cuda() for _, Y in obs]

    def loss(Xb0, logr, lam):
        X, L = Xb0, 0.0
        for t in range(CYCLES):
            Xa = enkfmc_analysis(X, logr, lam, plan, Ys[t])
            L = L + torch.sum((Xa - truths[t]) ** 2)
            X = _shift(Xa, p.geometry, 1)
        return L

    return p, obs, loss


def test_chain_gradient_matches_oracle(chain):
    p, obs, loss = chain
    Xb0 = torch.as_tensor(p.Xb).cuda().requires_grad_(True)
    logr = torch.log(torch.as_tensor(p.r_diag)).cuda().requires_grad_(True)
    lam = torch.tensor(p.ridge, dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss(Xb0, logr, lam)
    L.backward()
    # oracle: forward chain, then the reverse chain over its per-cycle adjoint
    X = np.asarray(p.Xb, np.float64)
    saved = []
    for t in range(CYCLES):
        res = A.analyze(p.geometry, X, obs[t][1], p.obs_idx, p.r_diag, p.ridge)
        saved.append((X, res))
        X = synth.linear_forecast(res.Xa, p.geometry, 1)
    _say("[cycles] oracle forward done")
    gX = np.zeros_like(X)
    dlogR = np.zeros(p.m)
    dlam = 0.0
    for t in reversed(range(CYCLES)):
        Xt, res = saved[t]
        G = 2.0 * (res.Xa - obs[t][0][:, None]) + synth.linear_forecast(gX, p.geometry, -1)
        gX, dr, dl = J.analyze_backward(Xt, p.obs_idx, p.r_diag, p.ridge, res, G)
        dlogR += dr
        dlam += dl
    L_o = sum(float(np.sum((saved[t][1].Xa - obs[t][0][:, None]) ** 2)) for t in range(CYCLES))
    e = [abs(float(L) - L_o) / L_o,
         float(np.linalg.norm(Xb0.grad.cpu().numpy() - gX) / np.linalg.norm(gX)),
         float(np.linalg.norm(logr.grad.cpu().numpy() - dlogR) / np.linalg.norm(dlogR)),
         abs(float(lam.grad) - dlam) / abs(dlam)]
    _say(f"[cycles] L={float(L):.10e} oracle {L_o:.10e}; rel err L {e[0]:.2e} dX_b {e[1]:.2e} "
         f"dlog r {e[2]:.2e} dlam {e[3]:.2e}")
    assert e[0] <= 1e-6 and max(e[1:]) <= 1e-5


def test_chain_gradient_matches_finite_differences(chain):
    p, obs, loss = chain
    Xb0 = torch.as_tensor(p.Xb).cuda().requires_grad_(True)
    logr = torch.log(torch.as_tensor(p.r_diag)).cuda().requires_grad_(True)
    lam = torch.tensor(p.ridge, dtype=torch.float64, device="cuda", requires_grad=True)
    loss(Xb0, logr, lam).backward()
    g = np.random.default_rng(21)

    def richardson(f, h):
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    X0, r0, l0 = Xb0.detach(), logr.detach(), lam.detach()
    with torch.no_grad():
        for _ in range(8):   # eight random directions per parameter group
            V = torch.as_tensor(g.standard_normal(p.Xb.shape)).cuda()
            fd = richardson(lambda e: float(loss(X0 + e * V, r0, l0)), 1e-4)
            ad = float(torch.sum(Xb0.grad * V))
            _say(f"[cycles fd] X_b: fd={fd:.10e} adjoint={ad:.10e}")
            assert abs(fd - ad) <= 1e-6 * abs(fd)
            v = torch.as_tensor(g.standard_normal(p.m)).cuda()
            fd = richardson(lambda e: float(loss(X0, r0 + e * v, l0)), 1e-4)
            ad = float(torch.sum(logr.grad * v))
            _say(f"[cycles fd] log r: fd={fd:.10e} adjoint={ad:.10e}")
            assert abs(fd - ad) <= 1e-6 * abs(fd)
        fd = richardson(lambda e: float(loss(X0, r0, l0 + e)), 1e-6)
        _say(f"[cycles fd] lam: fd={fd:.10e} adjoint={float(lam.grad):.10e}")
        assert abs(fd - float(lam.grad)) <= 1e-6 * abs(fd)
