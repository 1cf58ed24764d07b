"""isis_mg: FAS multigrid for the symmetron / Hu-Sawicki f(R) scalar-field
equation (Llinares, Mota & Winther 2013) on one MI355X.

The compute path is the HIP library libisis_mg.so (C ABI in
include/isis_mg.h); this package only marshals torch tensors into it.
Importing the package does not load the library; the first solver call does,
and fails loudly if it has not been built.
"""
from . import synth  # noqa: F401

__all__ = ["synth", "Solver", "ModelParams", "symmetron", "fofr", "linear", "IsisError",
           "NotConverged", "Diverged"]


def __getattr__(name):
    if name in ("Solver", "ModelParams", "symmetron", "fofr", "linear", "IsisError",
                "NotConverged", "Diverged", "Stats"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
