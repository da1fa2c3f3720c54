"""MI355X (gfx950) split-step solver for the two-component quasi-2D Gross-Pitaevskii equation.

The compute path is the HIP library libsgpe.so (C ABI in include/sgpe.h); this package is its
thin Python binding.  Build it with ``python -m paper_2010_15069_amd.build``.
"""
from ._lib import LIB_PATH, SgpeError, SgpeParams, STATUS_NAMES
from .solver import Batch, Solver, device_count, probe_exchange, probe_placement, validate_params

__all__ = ["Batch", "Solver", "SgpeError", "SgpeParams", "STATUS_NAMES", "LIB_PATH", "device_count",
           "probe_exchange", "probe_placement", "validate_params"]
