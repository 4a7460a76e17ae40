"""MI355X (gfx950) library for the per-time-step solve of the CN / SIPG-PolyDG
monodomain system with the two-level additive Schwarz PCG (arXiv 2512.19536).

The compute path is libpdg.so (hand-written HIP kernels + C++ setup) behind the
C-ABI in include/pdg.h; this package only marshals arguments to it.
"""
from ._lib import EXPORTS, PdgError, load  # noqa: F401
from .solver import BatchSolver, Context, from_problem, initial_state, step_batch  # noqa: F401

__all__ = ["Context", "from_problem", "initial_state", "PdgError", "load", "EXPORTS"]
