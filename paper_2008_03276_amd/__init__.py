"""MI355X (gfx950) PAQIF / EHL library: Python binding.

The numerical work runs in ``libpaqif_ehl.so`` (hand-written HIP); this
package marshals torch tensors into its C ABI (``include/paqif_ehl.h``).
"""
from . import _binding
from ._binding import (LCP_CLIP, LCP_EXACT, LCP_EXACT_FROM_U, LCP_LINEAR, PREC_FP32, PREC_FP32_IR, PREC_FP64,
                       PREC_SPLIT_BF16, SYS_LCP_NOT_CONVERGED, SYS_NEGATIVE_FILM,
                       SYS_NEWTON_NOT_CONVERGED, SYS_NONFINITE, SYS_OK, SYS_REFINE_STALLED,
                       SYS_ZERO_PIVOT, LibraryMissing, lib)
from . import paqif
from . import ehl
from . import convdiff

__all__ = ["lib", "paqif", "ehl", "convdiff", "LibraryMissing"]
