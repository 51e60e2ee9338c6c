"""MI355X (gfx950) library for the matrix-free elastic Lippmann-Schwinger
solve and the Frechet / adjoint operators of the distorted-Born method
(Xiang et al., arXiv 2402.02116).

The compute path is libfwils.so (hand-written HIP kernels behind the C ABI
declared in include/fwils.h); this package is its Python binding.  There is
no CPU fallback: without the built library or a GPU, calls raise.
"""

from ._lib import FwilsError, FwilsLibraryError, load  # noqa: F401

__all__ = ["Plan", "FrechetFn", "FrechetOperator", "LaplacianFn", "tikhonov_loss", "load", "FwilsError",
           "FwilsLibraryError"]


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name in ("FrechetFn", "FrechetOperator", "LaplacianFn", "tikhonov_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
