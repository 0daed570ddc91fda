"""Python face of the EnKF-MC library: a Plan over one geometry and observation
network.  torch supplies device memory and the current HIP stream; every step
of the hot path runs inside libenkfmc.so."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Tuple

import numpy as np

from . import _lib
from ._lib import EnkfmcError, F32, F64, FIT_BATCHED, FIT_PLAIN, FIT_SVD, SOLVE_DUAL, SOLVE_PCG, check  # noqa: F401

_MODES = {"plain": FIT_PLAIN, "batched": FIT_BATCHED, "svd": FIT_SVD}
_SOLVERS = {"dual": SOLVE_DUAL, "pcg": SOLVE_PCG}


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def analysis_sq_error_noalloc(Xa, x_ref, err=None):
    """sum_g (mean_k X_a[g, k] - x_ref[g])^2 through the allocation-free entry
    point (no plan, no workspace; the library's static scratch).  Xa (n, N)
    float32/float64 CUDA with unit member stride, x_ref (n,) float64 CUDA
    contiguous; err: a (1,) float64 CUDA tensor to write (allocated here when
    None).  The call only enqueues its kernels on the current stream."""
    import torch
    lib = _lib.load()
    p, dt, ld = Plan._xb_args(Xa)
    n, N = int(Xa.shape[0]), int(Xa.shape[1])
    if (x_ref.dtype != torch.float64 or not x_ref.is_cuda or not x_ref.is_contiguous()
            or tuple(x_ref.shape) != (n,)):
        raise ValueError("x_ref must be a contiguous float64 CUDA tensor of n elements")
    if err is None:
        err = torch.empty((1,), dtype=torch.float64, device=Xa.device)
    check(lib.enkfmc_analysis_sq_error_noalloc(n, N, p, dt, ld, ctypes.c_void_p(x_ref.data_ptr()),
                                               ctypes.c_void_p(err.data_ptr()),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return err


def timestamp(slot) -> None:
    """Enqueue a write of the device wall clock into `slot` (a one-element
    int64 CUDA tensor or a view of one) on the current stream."""
    import torch
    if slot.dtype != torch.int64 or not slot.is_cuda or slot.numel() != 1:
        raise ValueError("slot must be a one-element int64 CUDA tensor")
    check(_lib.load().enkfmc_timestamp(ctypes.c_void_p(slot.data_ptr()),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def wall_clock_hz() -> int:
    """Rate of the device wall clock that timestamp() reads."""
    hz = ctypes.c_int64()
    check(_lib.load().enkfmc_wall_clock_hz(ctypes.byref(hz)))
    return int(hz.value)


class Plan:
    """Decomposition of one geometry (Section 3) plus its device workspace.

    geometry: dict(nx, ny, nlev=[...], periodic_x, sdx, sdy, r_h, r_v)
    N: ensemble size; obs_idx: observed components (strictly increasing).
    """

    def __init__(self, geometry: Dict, N: int, obs_idx):
        self.lib = _lib.load()
        self.geometry = dict(geometry)
        nlev = np.ascontiguousarray(np.asarray(geometry["nlev"], dtype=np.int32))
        self._nlev = nlev
        g = _lib.Geometry(int(geometry["nx"]), int(geometry["ny"]), int(nlev.size), _ptr(nlev, ctypes.c_int32),
                          int(geometry["periodic_x"]), int(geometry["sdx"]), int(geometry["sdy"]),
                          int(geometry["r_h"]), int(geometry["r_v"]))
        obs = np.ascontiguousarray(np.asarray(obs_idx, dtype=np.int32))
        self.obs_idx = obs
        h = ctypes.c_void_p()
        check(self.lib.enkfmc_plan_create(ctypes.byref(h), ctypes.byref(g), int(N), _ptr(obs, ctypes.c_int32),
                                          int(obs.size)))
        self._h = h
        self.N = int(N)
        info = _lib.PlanInfo()
        check(self.lib.enkfmc_plan_get_info(self._h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _lib.PlanInfo._fields_}
        self.workspace = None

    # ------------------------------------------------------------------ host
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.enkfmc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()
        self.workspace = None
        self._factor_cache = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self) -> int:
        return int(self.info["n"])

    @property
    def m(self) -> int:
        return int(self.info["m"])

    def pattern(self, k: int) -> Dict[str, np.ndarray]:
        n_sd, nnz, m_sd = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(self.lib.enkfmc_get_pattern_sizes(self._h, int(k), ctypes.byref(n_sd), ctypes.byref(nnz),
                                                ctypes.byref(m_sd)))
        out = dict(loc2glob=np.empty(n_sd.value, np.int64), interior=np.empty(n_sd.value, np.uint8),
                   row_ptr=np.empty(n_sd.value + 1, np.int64), col_idx=np.empty(nnz.value, np.int32),
                   obs=np.empty(m_sd.value, np.int32), obs_row=np.empty(m_sd.value, np.int32))
        check(self.lib.enkfmc_get_pattern(self._h, int(k), _ptr(out["loc2glob"], ctypes.c_int64),
                                          _ptr(out["interior"], ctypes.c_uint8), _ptr(out["row_ptr"], ctypes.c_int64),
                                          _ptr(out["col_idx"], ctypes.c_int32), _ptr(out["obs"], ctypes.c_int32),
                                          _ptr(out["obs_row"], ctypes.c_int32)))
        return out

    def row_counts(self, k: int) -> np.ndarray:
        """Predecessor count of every local row of sub-domain k."""
        n_sd = ctypes.c_int64()
        check(self.lib.enkfmc_get_pattern_sizes(self._h, int(k), ctypes.byref(n_sd), None, None))
        rp = np.empty(n_sd.value + 1, np.int64)
        check(self.lib.enkfmc_get_pattern(self._h, int(k), None, None, _ptr(rp, ctypes.c_int64), None, None, None))
        return np.diff(rp)

    def set_timing(self, enable: bool = True) -> None:
        check(self.lib.enkfmc_set_timing(self._h, 1 if enable else 0))

    def set_async(self, enable: bool = True) -> None:
        """Calls only enqueue their kernels (no status read, no memset), so
        that several plans run concurrently and calls can be captured into a
        HIP graph; check_status() reads the accumulated device status."""
        check(self.lib.enkfmc_set_async(self._h, 1 if enable else 0))

    def check_status(self) -> None:
        """Synchronise the current stream and raise the first device-side
        failure recorded since the last check (asynchronous mode)."""
        check(self.lib.enkfmc_check_status(self._h, self._stream()))

    def timing(self) -> Dict[str, float]:
        out = {}
        for i, name in enumerate(_lib.PHASES):
            v = ctypes.c_double()
            check(self.lib.enkfmc_get_timing(self._h, i, ctypes.byref(v)))
            out[name] = v.value
        return out

    # ---------------------------------------------------------------- device
    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def ensure_workspace(self):
        import torch
        if self.workspace is None:
            nbytes = int(self.info["workspace_bytes"])
            self.workspace = torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device="cuda")
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            check(self.lib.enkfmc_plan_set_workspace(self._h, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                                                     self._stream()))
        return self.workspace

    def set_factor_cache(self, enable: bool = True) -> int:
        """Keep the regressions' Cholesky tiles from each batched fit in
        device memory owned by this object, so that the reverse pass reads
        them instead of recomputing each row's Gram and factorisation.
        Returns the bytes held (0 when disabled)."""
        import torch
        check(self.lib.enkfmc_plan_set_factor_cache(self._h, None, ctypes.c_size_t(0)))
        self._factor_cache = None
        if not enable:
            return 0
        nbytes = int(self.info["factor_cache_bytes"])
        if nbytes == 0:
            return 0
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (buf.data_ptr() + 255) & ~255
        check(self.lib.enkfmc_plan_set_factor_cache(self._h, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes)))
        self._factor_cache = buf
        return nbytes

    @staticmethod
    def _xb_args(Xb):
        import torch
        if Xb.dim() != 2 or not Xb.is_cuda or Xb.stride(1) != 1:
            raise ValueError("Xb must be a (n, N) CUDA tensor with unit member stride")
        if Xb.dtype == torch.float32:
            dt = F32
        elif Xb.dtype == torch.float64:
            dt = F64
        else:
            raise ValueError("Xb must be float32 or float64")
        return ctypes.c_void_p(Xb.data_ptr()), dt, Xb.stride(0)

    def fit(self, Xb, ridge: float = 0.0, mode: str = "batched") -> None:
        """eq. (1)/(8) in every sub-domain; T and D stay in the workspace."""
        self.ensure_workspace()
        self._check_xb(Xb)
        p, dt, ld = self._xb_args(Xb)
        self._token = getattr(self, "_token", 0) + 1
        check(self.lib.enkfmc_fit(self._h, p, dt, ld, float(ridge), _MODES[mode], self._stream()))

    def set_pcg(self, maxit: int = 2000, rtol: float = 1e-12) -> None:
        """Iteration limit and relative tolerance of solver="pcg"."""
        check(self.lib.enkfmc_set_pcg(self._h, int(maxit), float(rtol)))

    def pcg_stats(self) -> Dict:
        """Iterations, largest per-column count, refinement restarts and the
        largest final relative residual of the last PCG analysis."""
        it, mc, rf = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rr = ctypes.c_double()
        check(self.lib.enkfmc_get_pcg_stats(self._h, ctypes.byref(it), ctypes.byref(mc), ctypes.byref(rf),
                                            ctypes.byref(rr), self._stream()))
        return {"iterations": it.value, "max_column_iterations": mc.value, "refinements": rf.value,
                "max_rel_residual": rr.value}

    def analyze(self, Xb, Y, r_diag, out_dtype=None, solver: str = "dual"):
        """Local analyses + merge (eq. 11/14, Alg. 2-3).  Returns X_a (n, N).
        solver: "dual" (eqs. 12-13, direct) or "pcg" (primal eq. 11 by
        B^-preconditioned conjugate gradients)."""
        import torch
        self._check_xb(Xb)
        Y = self._dev64(Y, (self.m, self.N), "Y")
        r = self._dev64(r_diag, (self.m,), "r_diag")
        out_dtype = out_dtype or torch.float64
        Xa = torch.empty((self.n, self.N), dtype=out_dtype, device=Xb.device)
        p, dt, ld = self._xb_args(Xb)
        self._analysis_inputs = None
        self._token = getattr(self, "_token", 0) + 1
        check(self.lib.enkfmc_analyze(self._h, p, dt, ld, ctypes.c_void_p(Y.data_ptr()),
                                      ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(Xa.data_ptr()),
                                      F32 if out_dtype == torch.float32 else F64, _SOLVERS[solver],
                                      self._stream()))
        # the reverse pass reads the same device copies of Y and r_diag
        self._analysis_inputs = (Y, r)
        return Xa

    @property
    def analysis_token(self) -> int:
        """Changes with every fit and analysis; a reverse pass is valid only
        while it equals the value read right after the matching analyze."""
        return getattr(self, "_token", 0)

    def backward(self, Xb, dXa) -> Tuple:
        """dL/dX_b, dL/dlog r, dL/dridge from dL/dX_a, for the preceding
        fit + analyze of this plan on the same X_b (derivation in
        csrc/backward.hip)."""
        import torch
        self._check_xb(Xb)
        if getattr(self, "_analysis_inputs", None) is None:
            raise EnkfmcError(-7, "backward: needs the preceding fit + analyze")
        Y, r = self._analysis_inputs
        g = self._dev64(dXa, (self.n, self.N), "dXa")
        dXb = torch.empty((self.n, self.N), dtype=torch.float64, device=Xb.device)
        dlogR = torch.empty((max(self.m, 1),), dtype=torch.float64, device=Xb.device)
        dridge = torch.empty((1,), dtype=torch.float64, device=Xb.device)
        p, dt, ld = self._xb_args(Xb)
        check(self.lib.enkfmc_analyze_backward(self._h, p, dt, ld, ctypes.c_void_p(Y.data_ptr()),
                                               ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                               ctypes.c_void_p(dXb.data_ptr()), ctypes.c_void_p(dlogR.data_ptr()),
                                               ctypes.c_void_p(dridge.data_ptr()), self._stream()))
        return dXb, dlogR[:self.m], dridge[0]

    def perturb_observations(self, y, r_diag, seed: int, cycle: int, out=None):
        """Y^s = y 1^T + E of one assimilation time (Alg. 1), E drawn on the
        device from N(0, R) by the counter-based generator of
        include/enkfmc.h.  Returns (m, N) float64 (`out` if given)."""
        import torch
        if self.m == 0:
            return torch.empty((0, self.N), dtype=torch.float64, device="cuda")
        self.ensure_workspace()
        yv = self._dev64(y, (self.m,), "y")
        r = self._dev64(r_diag, (self.m,), "r_diag")
        if out is None:
            out = torch.empty((max(self.m, 1), self.N), dtype=torch.float64, device="cuda")
        elif (out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous()
              or out.numel() < self.m * self.N):
            raise ValueError("out must be a contiguous float64 CUDA tensor of m x N elements")
        check(self.lib.enkfmc_perturb_observations(self._h, ctypes.c_void_p(yv.data_ptr()),
                                                   ctypes.c_void_p(r.data_ptr()), int(seed) & (2**64 - 1),
                                                   int(cycle) & (2**64 - 1), ctypes.c_void_p(out.data_ptr()),
                                                   self._stream()))
        return out[:self.m] if out.dim() == 2 else out

    def analysis_sq_error(self, Xa, x_ref):
        """sum_g (mean_k X_a[g, k] - x_ref[g])^2 (the summand of eq. 18), as a
        (1,) float64 device tensor."""
        import torch
        self.ensure_workspace()
        self._check_xb(Xa)
        p, dt, ld = self._xb_args(Xa)
        xr = self._dev64(x_ref, (self.n,), "x_ref")
        err = torch.empty((1,), dtype=torch.float64, device="cuda")
        check(self.lib.enkfmc_analysis_sq_error(self._h, p, dt, ld, ctypes.c_void_p(xr.data_ptr()),
                                                ctypes.c_void_p(err.data_ptr()), self._stream()))
        return err

    def factors(self, k: int):
        n_sd, nnz, _ = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(self.lib.enkfmc_get_pattern_sizes(self._h, int(k), ctypes.byref(n_sd), ctypes.byref(nnz), None))
        tval = np.empty(nnz.value, np.float64)
        d = np.empty(n_sd.value, np.float64)
        check(self.lib.enkfmc_get_factors(self._h, int(k), _ptr(tval, ctypes.c_double), _ptr(d, ctypes.c_double),
                                          self._stream()))
        return tval, d

    def increment(self, k: int) -> np.ndarray:
        n_sd = ctypes.c_int64()
        check(self.lib.enkfmc_get_pattern_sizes(self._h, int(k), ctypes.byref(n_sd), None, None))
        Z = np.empty((n_sd.value, self.N), np.float64)
        check(self.lib.enkfmc_get_increment(self._h, int(k), _ptr(Z, ctypes.c_double), self._stream()))
        return Z

    # ---------------------------------------------------------------- checks
    def _check_xb(self, Xb):
        if tuple(Xb.shape) != (self.n, self.N):
            raise ValueError(f"Xb has shape {tuple(Xb.shape)}, expected {(self.n, self.N)}")

    def _dev64(self, t, shape, name):
        import torch
        if self.m == 0 and name in ("Y", "r_diag"):
            return torch.zeros(1, dtype=torch.float64, device="cuda")
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.asarray(t))
        t = t.to(device="cuda", dtype=torch.float64).contiguous()
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return t
