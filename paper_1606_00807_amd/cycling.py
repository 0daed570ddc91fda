"""Assimilation cycles (Alg. 1) and the RMSE of eq. (18).

Each assimilation time t draws the perturbed observations Y^s of y_t on the
device, fits B^-1 on the current background, runs the analysis, records the
squared error of the analysis mean against the reference state (if one is
given), and hands the analysis ensemble to the forecast model for the next
background.  The forecast model is the caller's (the method does not include
one); every other step runs in libenkfmc.so.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

from . import _lib
from .api import Plan


@dataclass
class CycleResult:
    Xa: object                 # analysis ensemble of the last assimilation time (n, N)
    sq_err: Optional[object]   # (M,) float64 device tensor of ||mean(X_a^t) - x_ref^t||^2, or None
    rmse: Optional[float]      # eq. (18), or None without reference states


def rmse(sq_err) -> float:
    """eq. (18): sqrt of the mean over the M assimilation times of the squared
    error of the analysis mean, computed by the library (enkfmc_rmse) from a
    CUDA tensor (or a sequence, copied to the device) of the M squared errors."""
    import torch
    sq = torch.as_tensor(sq_err, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
    if sq.numel() == 0:
        raise ValueError("rmse needs at least one assimilation time")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    _lib.check(_lib.load().enkfmc_rmse(ctypes.c_void_p(sq.data_ptr()), sq.numel(), ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return float(out.item())


def assimilate(plan: Plan, Xb, observations: Sequence, r_diag, ridge: float,
               forecast: Callable, seed: int, x_ref: Optional[Sequence] = None,
               mode: str = "batched", first_cycle: int = 0) -> CycleResult:
    """Alg. 1 over M = len(observations) assimilation times.

    Xb: (n, N) CUDA background ensemble of the first time.
    observations: y_t, (m,) each.  r_diag: (m,) observation error variances.
    forecast: maps the analysis ensemble of time t to the background of t + 1
    (not called after the last time).  seed, first_cycle: the perturbations of
    time t are drawn with cycle number first_cycle + t.
    x_ref: optional reference states (n,) per time for eq. (18).
    """
    import torch
    M = len(observations)
    if M == 0:
        raise ValueError("no observations to assimilate")
    if x_ref is not None and len(x_ref) != M:
        raise ValueError("x_ref needs one reference state per assimilation time")
    Ys = torch.empty((max(plan.m, 1), plan.N), dtype=torch.float64, device="cuda")
    errs: List = []
    X = Xb
    Xa = None
    for t in range(M):
        Y = plan.perturb_observations(observations[t], r_diag, seed, first_cycle + t, out=Ys)
        plan.fit(X, ridge, mode=mode)
        Xa = plan.analyze(X, Y, r_diag, out_dtype=X.dtype)
        if x_ref is not None:
            errs.append(plan.analysis_sq_error(Xa, x_ref[t]))
        if t + 1 < M:
            X = forecast(Xa)
    if x_ref is None:
        return CycleResult(Xa, None, None)
    sq = torch.cat(errs)
    return CycleResult(Xa, sq, rmse(sq))
