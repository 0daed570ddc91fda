"""The allocation-free squared error (enkfmc_analysis_sq_error_noalloc): no
plan, no workspace, a static device scratch.  Checked against the entry point
that takes the plan's workspace (same kernels, so the same bits) and against
the plain definition, on two calls in a row, the second on a smaller input
whose partial sums must not keep anything of the first call's."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_1606_00807_amd import Plan, _lib
from paper_1606_00807_amd.api import analysis_sq_error_noalloc

pytestmark = pytest.mark.gpu


def _case(nx, ny, nlev, N, dtype, seed):
    geo = synth.geometry(nx, ny, nlev, True, 2, 2, 1, 1)
    n = synth.state_size(geo)
    g = np.random.default_rng(seed)
    Xa = g.standard_normal((n, N)) * 3.0 + 1.0
    x_ref = g.standard_normal(n)
    plan = Plan(geo, N, np.arange(0, n, 7))
    return plan, torch.as_tensor(Xa.astype(dtype)).cuda(), torch.as_tensor(x_ref).cuda(), Xa.astype(dtype), x_ref


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_matches_workspace_entry_twice(dtype):
    big = _case(48, 24, [3], 40, dtype, 11)
    small = _case(12, 10, [1], 21, dtype, 12)
    got = []
    for plan, Xa, xr, Xa_h, xr_h in (big, small):
        print(f"noalloc sq error: n={plan.n} N={plan.N} dtype={np.dtype(dtype).name}", flush=True)
        e_ws = plan.analysis_sq_error(Xa, xr)
        e_na = analysis_sq_error_noalloc(Xa, xr)
        torch.cuda.synchronize()
        a, b = float(e_ws.item()), float(e_na.item())
        ref = float(np.sum((Xa_h.astype(np.float64).mean(1) - xr_h) ** 2))
        assert b == a, (b, a)                       # same kernels, same order: same bits
        assert abs(b - ref) <= 1e-12 * ref, (b, ref)
        got.append(b)
    assert got[0] != got[1]


def test_noalloc_rejects_bad_sizes():
    lib = _lib.load()
    Xa = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    xr = torch.zeros(4, dtype=torch.float64, device="cuda")
    err = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (ctypes.c_void_p(Xa.data_ptr()), _lib.F64, 3, ctypes.c_void_p(xr.data_ptr()),
            ctypes.c_void_p(err.data_ptr()), s)
    assert lib.enkfmc_analysis_sq_error_noalloc(2**31, 3, *args) == -8      # n beyond the limit
    assert "exceed" in lib.enkfmc_last_error().decode()
    assert lib.enkfmc_analysis_sq_error_noalloc(4, 70000, args[0], _lib.F64, 70000, *args[3:]) == -8  # N beyond
    assert lib.enkfmc_analysis_sq_error_noalloc(-1, 3, *args) == -1
    assert lib.enkfmc_analysis_sq_error_noalloc(4, 3, None, _lib.F64, 3, ctypes.c_void_p(xr.data_ptr()),
                                                ctypes.c_void_p(err.data_ptr()), s) == -1
    # n = 0: the sum is empty
    assert lib.enkfmc_analysis_sq_error_noalloc(0, 3, *args) == 0
    torch.cuda.synchronize()
    assert float(err.item()) == 0.0
