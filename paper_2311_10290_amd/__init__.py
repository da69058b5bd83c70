"""MI355X loop-erased-walk estimators of the Laplacian pseudo-inverse.

Thin Python binding over the C ABI in ``include/lap.h`` (``liblap.so``,
hand-written HIP for gfx950).  Every step of the hot path runs in the
library's kernels; this package only marshals arguments.  Importing it
without the built library raises ``ImportError`` -- there is no fallback.
"""
from .api import (LapError, Graph, Batch, Server, load_library, prof_enable, prof_read, prof_reset,  # noqa: F401
                  diag_Ldagger, ecc, kemeny, bench_gather)
