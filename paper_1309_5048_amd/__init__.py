"""MI355X (gfx950) solver for the divergence-conforming B-spline Stokes system by
block-diagonally preconditioned MINRES (Cortes & Coutinho, arXiv 1309.5048).

The compute path is libstokes.so (hand-written HIP kernels behind the C ABI of
include/stokes.h); this package is its Python binding.
"""
from ._native import (CAVITY_LID, CAVITY_VERIFY, FP64, GEOMETRY_ANNULUS, GEOMETRY_SQUARE, MIXED, PC_IC0, PC_ICPCG, PC_ICPCG_AQ, PC_IDEAL,  # noqa: F401
                      PC_IDEAL_A, PC_JACOBI, PC_JPCG, PC_PCGAQ, LIB_PATH)


def __getattr__(name):
    # torch-dependent parts are imported lazily
    if name in ("StokesProblem", "StokesError"):
        from . import solver
        return getattr(solver, name)
    if name in ("StokesSolve", "stokes_solve"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
