"""MI355X-native soft-force hot path of the P3T scheme with individual
cut-off radii (Ishigaki et al. 2021, GPLUM).

libp3t.so (HIP kernels for gfx950 behind the C ABI of include/p3t.h) does all
the computing; this package is its Python binding.  Import is cheap: the
library is loaded on first use and a missing library is an error.
"""
from ._lib import LIB_PATH, load  # noqa: F401
from .api import Context, P3TError, Params, compute_cutoffs_noalloc  # noqa: F401

__all__ = ["load", "LIB_PATH", "Context", "Params", "P3TError", "compute_cutoffs_noalloc"]
