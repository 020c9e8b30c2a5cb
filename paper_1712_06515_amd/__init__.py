"""MI355X (gfx950) resampled cross-correlation: rho for every orbital template and bin.

The computation lives in ``libccr.so`` (C ABI in include/ccr.h); ``ccr`` is its binding.
"""

from .ccr import (  # noqa: F401
    Context, CcrError, load_library, LIB_PATH, PREC_FP64, PREC_SPLIT, PAIRS_CROSS, PAIRS_SAME,
)
