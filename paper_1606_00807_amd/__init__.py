"""MI355X-native EnKF based on the modified Cholesky decomposition (arXiv 1606.00807).

The hot path (sub-domain fit of B^-1 = T^T D^-1 T and local analyses) lives in
libenkfmc.so (hand-written HIP for gfx950, C ABI in include/enkfmc.h).  This
package is its thin binding: ``Plan`` (api.py) and the autograd wrapper.
"""
from .api import EnkfmcError, Plan  # noqa: F401
from .autograd import EnkfmcAnalysis, enkfmc_analysis  # noqa: F401
