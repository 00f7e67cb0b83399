"""MI355X-native dense revised simplex (explicit B^-1) behind the lpgpu C ABI.

The product path is liblpgpu.so (HIP kernels for gfx950 + C runtime); this package
only loads it and marshals arguments.  See include/lpgpu.h for the ABI.
"""
from .binding import (LP, Batch, LP_FP64, LP_INFEASIBLE, LP_ITER_LIMIT, LP_MAX, LP_MIN, LP_MIXED, LP_NUMERICAL,
                      LP_OPTIMAL, LP_PIVOT_DRIVEOUT, LP_ROW_EQ, LP_ROW_GE, LP_ROW_LE, LP_RUNNING, LP_UNBOUNDED,
                      LPError, STATUS_NAMES, default_options, lib, solve_device_noalloc)

__all__ = ["LP", "Batch", "LPError", "default_options", "lib", "LP_OPTIMAL", "LP_UNBOUNDED", "LP_ITER_LIMIT", "LP_NUMERICAL",
           "LP_INFEASIBLE", "LP_RUNNING", "LP_MAX", "LP_MIN", "LP_FP64", "LP_MIXED", "LP_ROW_LE", "LP_ROW_GE",
           "LP_ROW_EQ", "LP_PIVOT_DRIVEOUT", "STATUS_NAMES", "solve_device_noalloc"]
