"""Plain, slow, FP64 CPU oracle of the EnKF-MC hot path (arXiv 1606.00807).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (its own decomposition, its own regression, its own solves).

Modules
-------
geometry  sub-domain decomposition, local ordering, radius-restricted
          predecessors and local observation lists (Section 3, Fig. 2 text,
          Alg. 2 decomposition steps).
fit       ensemble anomalies (eq. 5) and the modified-Cholesky regression of
          every local component on its predecessors (eq. 1, eq. 8).
analysis  local primal analysis solved directly (eq. 11 per sub-domain, eq. 14,
          Alg. 3) and mapped back on interior rows (Alg. 2 merge step); the
          dual form (eqs. 12-13) as an independent cross-check.
adjoint   reverse-mode derivative of fit + analysis with respect to X_b,
          log diag(R) and the ridge parameter.
cycling   perturbed observations (Section 2.3, Alg. 1) from a counter-based
          generator, the cycle loop of Alg. 1 and the RMSE of eq. (18).

Every floating-point computation is in float64.  Readings of points where the
paper is silent or ambiguous are listed in the module docstrings (R1..R14).
"""

from . import geometry, fit, analysis, adjoint, cycling  # noqa: F401
from .errors import OracleError  # noqa: F401
