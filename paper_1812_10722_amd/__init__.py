"""MI355X-native quasistatic LSPR boundary-element solver (treecode + batched GMRES in HIP).

The compute lives in liblspr.so (C ABI in include/lspr.h); `lspr` is its thin binding.
"""
from . import lspr  # noqa: F401  (raises ImportError when the HIP library is not built)
from .lspr import Geometry, op_params, gmres_params, LsprError  # noqa: F401
