"""Fast directional Helmholtz matvec on MI355X (gfx950).

The library ``libfdm.so`` (C ABI in ``include/fdm.h``) implements the fast
directional matrix-vector product of Of & Watschinger (uniform box cluster
trees, directional Chebyshev interpolation, Alg. 4) in hand-written HIP; this
package is its thin Python binding.
"""
from .fdm import (Batch, Plan, FdmError, aca, dense_matvec, lib, header_functions, PRECISION,
                  STATUS, LIB_PATH)

__all__ = ["Batch", "Plan", "FdmError", "aca", "dense_matvec", "lib", "header_functions",
           "PRECISION", "STATUS", "LIB_PATH"]
