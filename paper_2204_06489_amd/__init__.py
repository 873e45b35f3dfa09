"""MI355X-native full-space Gauss-Newton KKT solver for 2-D frequency-domain FWI.

Implements the Newton-step KKT system of arXiv 2204.06489 (Sections 2-5): the
matrix-free KKT operator, the block-triangular preconditioner and its
inexact-block variant, batched Helmholtz A / A^H block solves over all
sources, flexible GMRES and the Gauss-Newton update, as HIP kernels for gfx950
behind the C ABI in include/kktfwi.h.  This package is the Python binding.
"""

from ._lib import KFError, LIB_PATH, header_functions, lib  # noqa: F401

__all__ = ["KFError", "LIB_PATH", "header_functions", "lib", "KKTProblem", "HelmholtzSolve"]


def __getattr__(name):
    # torch is imported lazily so that the C ABI checks work without it
    if name == "KKTProblem":
        from .solver import KKTProblem
        return KKTProblem
    if name == "HelmholtzSolve":
        from .autograd import HelmholtzSolve
        return HelmholtzSolve
    raise AttributeError(name)
