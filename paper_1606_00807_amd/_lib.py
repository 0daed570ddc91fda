"""ctypes binding of libenkfmc.so (argument marshalling only).

Every computation of the hot path runs in the library's HIP kernels; this
module only loads the shared object and declares the C signatures of
include/enkfmc.h.  It raises if the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint8, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libenkfmc.so")

ENKFMC_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "ENONPOS_D", -4: "ENOCONV", -5: "EHIP", -6: "ENOMEM",
          -7: "ESTATE", -8: "EUNSUPPORTED"}
F32, F64 = 0, 1
FIT_PLAIN, FIT_BATCHED, FIT_SVD = 0, 1, 2
SOLVE_DUAL, SOLVE_PCG = 0, 1
PHASES = ["anomaly", "fit", "dual_F", "dual_S", "dual_chol", "dual_Q", "dual_G", "sweep", "mapback", "backward",
          "tiles", "fit_kform",
          "adj_solve", "adj_factor", "adj_regress", "adj_gather", "fit_fallback", "pcg"]


class Geometry(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nvar", c_int32), ("nlev", POINTER(c_int32)),
                ("periodic_x", c_int32), ("sdx", c_int32), ("sdy", c_int32), ("r_h", c_int32), ("r_v", c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("N", c_int64), ("m", c_int64), ("n_subdomains", c_int64), ("n_blocks", c_int64),
                ("n_fit", c_int64), ("nnz", c_int64), ("m_local", c_int64), ("max_p", c_int32),
                ("max_block_rows", c_int32), ("max_block_obs", c_int32), ("reserved", c_int32),
                ("workspace_bytes", c_size_t), ("fit_rows_wave", c_int64), ("fit_rows_plain", c_int64),
                ("n_row_tiles", c_int64), ("n_tiles", c_int64), ("f_entries", c_int64), ("s_entries", c_int64),
                ("factor_cache_bytes", c_size_t), ("near_d", c_int32), ("far_lo", c_int32),
                ("max_tile_distance", c_int32), ("far_ring", c_int32)]


class EnkfmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.code = STATUS.get(status, str(status))


_LIB = None

SIGNATURES = {
    "enkfmc_plan_create": (c_int32, [POINTER(c_void_p), POINTER(Geometry), c_int32, POINTER(c_int32), c_int32]),
    "enkfmc_plan_get_info": (c_int32, [c_void_p, POINTER(PlanInfo)]),
    "enkfmc_plan_set_workspace": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "enkfmc_plan_set_factor_cache": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "enkfmc_fit": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_double, c_int32, c_void_p]),
    "enkfmc_analyze": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_int32,
                                 c_int32, c_void_p]),
    "enkfmc_analyze_backward": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p]),
    "enkfmc_perturb_observations": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint64, c_uint64, c_void_p,
                                              c_void_p]),
    "enkfmc_analysis_sq_error": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p]),
    "enkfmc_analysis_sq_error_noalloc": (c_int32, [c_int64, c_int32, c_void_p, c_int32, c_int64, c_void_p,
                                                   c_void_p, c_void_p]),
    "enkfmc_rmse": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p]),
    "enkfmc_get_pattern_sizes": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_int64),
                                           POINTER(c_int64)]),
    "enkfmc_get_pattern": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_uint8), POINTER(c_int64),
                                     POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "enkfmc_get_factors": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), c_void_p]),
    "enkfmc_get_increment": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_void_p]),
    "enkfmc_set_timing": (c_int32, [c_void_p, c_int32]),
    "enkfmc_set_async": (c_int32, [c_void_p, c_int32]),
    "enkfmc_set_pcg": (c_int32, [c_void_p, c_int32, c_double]),
    "enkfmc_get_pcg_stats": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_double), c_void_p]),
    "enkfmc_check_status": (c_int32, [c_void_p, c_void_p]),
    "enkfmc_timestamp": (c_int32, [c_void_p, c_void_p]),
    "enkfmc_wall_clock_hz": (c_int32, [POINTER(c_int64)]),
    "enkfmc_get_timing": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "enkfmc_status_string": (c_char_p, [c_int32]),
    "enkfmc_last_error": (c_char_p, []),
    "enkfmc_plan_destroy": (None, [c_void_p]),
}


def load(path: str = LIB_PATH):
    """Load libenkfmc.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(there is no fallback implementation)")
    # torch ships its own copy of the HIP runtime; load it first so that the
    # library binds to the same runtime instance that owns torch's memory.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def hip_stream_create() -> int:
    """A new non-blocking HIP stream at the default priority, created by the
    runtime the library is bound to; returns the raw hipStream_t."""
    lib = load()
    fn = lib.hipStreamCreateWithFlags
    fn.restype, fn.argtypes = ctypes.c_int, [POINTER(c_void_p), ctypes.c_uint]
    s = c_void_p()
    err = fn(ctypes.byref(s), 1)  # hipStreamNonBlocking
    if err != 0:
        raise RuntimeError(f"hipStreamCreateWithFlags failed ({err})")
    return int(s.value)


def hip_stream_destroy(stream: int) -> None:
    """Wait for the stream's work, then destroy it."""
    lib = load()
    sync, destroy = lib.hipStreamSynchronize, lib.hipStreamDestroy
    for fn in (sync, destroy):
        fn.restype, fn.argtypes = ctypes.c_int, [c_void_p]
    err = sync(c_void_p(stream)) or destroy(c_void_p(stream))
    if err != 0:
        raise RuntimeError(f"destroying a HIP stream failed ({err})")


def check(status: int) -> None:
    if status != ENKFMC_OK:
        msg = load().enkfmc_last_error().decode(errors="replace")
        raise EnkfmcError(status, msg)
