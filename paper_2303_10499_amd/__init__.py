"""MI355X (gfx950) implementation of one segregated pressure-based time step of
the dry compressible Euler equations (GEA, arXiv:2303.10499, Sec. 3) and of
its pressure solve: FP64 Jacobi-PCG, FP32/FP64 iterative refinement, and a
learned initial guess/preconditioner.  The compute path is the C-ABI library
``libgea.so`` (include/gea.h); ``gea`` is its Python binding.
"""
from . import configs  # noqa: F401

__all__ = ["configs", "gea", "build"]
