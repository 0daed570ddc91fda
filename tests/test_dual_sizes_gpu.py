"""GPU parity of the dual form's local solve at the block sizes that choose
its kernels (eqs. 12-13: S = R + H B H^T factored, then Q = S^-1 (Y^s - H X_b)).

Blocks of up to 128 observations factor S by 16 x 16 register tiles and solve
with it by 16-row tiles on the matrix cores; larger blocks take the one-lane
and workgroup kernels.  Each workload below is one sub-domain holding one
variable on one level, so its single block holds exactly m observations:
  m = 16    one full tile, no padding
  m = 113   eight tiles, the last padded to 128
  m = 128   eight full tiles, the largest the tile kernels take
  m = 129   one past them: the other kernels
The local increment (1e-8) and the reverse pass's gradients (1e-5, the
adjoint tests' tolerance) are checked against the FP64 oracle; both use the
factor of S (the reverse pass solves with it again).
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as J
from oracle import analysis as A
from paper_1606_00807_amd import Plan

pytestmark = pytest.mark.gpu

# (nx, ny, observed fraction) of a one-block workload with m = round(frac * nx * ny)
SIZES = {16: (16, 16, 0.0625), 113: (16, 16, 113 / 256), 128: (16, 16, 0.5), 129: (43, 6, 0.5)}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@pytest.mark.parametrize("m", sorted(SIZES))
def test_dual_solve_matches_oracle_at_block_size(m):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nx, ny, frac = SIZES[m]
    p = synth.make_small(nx=nx, ny=ny, nlev=(1,), N=24, r_h=1, r_v=1, sdx=1, sdy=1, obs_frac=frac, ridge=1e-3,
                         config=400 + m)
    assert p.m == m
    plan = Plan(p.geometry, p.N, p.obs_idx)
    assert plan.info["n_blocks"] == 1 and plan.info["max_block_obs"] == m
    _say(f"[dual sizes] m={m} n={p.n} N={p.N}")
    res = A.analyze(p.geometry, p.Xb, p.Y, p.obs_idx, p.r_diag, p.ridge)
    Xb = torch.as_tensor(p.Xb).cuda()
    plan.fit(Xb, p.ridge)
    Xa = plan.analyze(Xb, p.Y, p.r_diag).cpu().numpy()
    inc = float(np.linalg.norm(Xa - res.Xa) / np.linalg.norm(res.Xa - p.Xb))
    Gbar = 2.0 * (res.Xa - p.x_true[:, None])
    dXb_o, dlogR_o, dlam_o = J.analyze_backward(p.Xb, p.obs_idx, p.r_diag, p.ridge, res, Gbar)
    dXb, dlogR, dlam = plan.backward(Xb, torch.as_tensor(Gbar).cuda())
    torch.cuda.synchronize()
    e = (_rel2(dXb.cpu().numpy(), dXb_o), _rel2(dlogR.cpu().numpy(), dlogR_o), abs(float(dlam) - dlam_o) / abs(dlam_o))
    _say(f"[dual sizes] m={m} increment={inc:.2e} dXb={e[0]:.2e} dlogR={e[1]:.2e} dlam={e[2]:.2e}")
    assert inc <= 1e-8
    assert max(e) <= 1e-5
