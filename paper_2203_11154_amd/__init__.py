"""MI355X (gfx950) Vanka-type multigrid for the complex-shifted Laplacian
systems of diagonalisation-based parallel-in-time (ParaDIAG) methods
(He & Liu, arXiv 2203.11154).

The solver lives in the HIP library libvanka_mg.so (C ABI in
include/vanka_mg.h); this package only marshals torch tensors into it.
Importing the package does not load the library; the first solver object
does, and fails loudly if it has not been built.
"""
import importlib

__all__ = ["Grid", "VankaMG", "transform", "transform_noalloc", "transform_circulant", "lfa_omega", "ShiftedSolve", "ParaDiag", "inputs"]

_LAZY = {"Grid": "solver", "VankaMG": "solver", "transform": "solver", "transform_noalloc": "solver",
         "transform_circulant": "solver",
         "lfa_omega": "solver",
         "ShiftedSolve": "autograd", "ParaDiag": "autograd"}


def __getattr__(name):
    if name in _LAZY:
        return getattr(importlib.import_module(f"{__name__}.{_LAZY[name]}"), name)
    raise AttributeError(name)
