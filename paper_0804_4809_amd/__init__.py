"""libgeninv: Moore-Penrose inverse by full-rank Cholesky factorization on
AMD Instinct MI355X (gfx950).

Python binding of the C ABI declared in include/geninv.h.  The method is
P. Courrieu's (Section 2 and Appendix of "Fast Computation of Moore-Penrose
Inverse Matrices"): Gram matrix, full-rank Cholesky with strict pivot test,
inverse of L'L, product chain Y = L M M L' G'.
"""
from ._lib import GeninvError, LIB_PATH, load  # noqa: F401

__all__ = ["GeninvError", "LIB_PATH", "load", "api", "workloads"]


def __getattr__(name):
    # the torch-based API is imported lazily so that `workloads` and the
    # loader stay importable without initialising torch
    if name in ("api", "workloads"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
