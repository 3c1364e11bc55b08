"""MI355X (gfx950) implementation of the finite-element coarse-grid projection
(IFE-CGP) time step of Kashefi & Staples (Section 2.2, Eqs. 19-23).

Every step of the path runs in the HIP kernels of ``libcgp.so`` behind the C
ABI declared in ``include/cgp.h``.  This module only marshals arguments:
numpy arrays for host inputs, torch CUDA tensors (HIP under ROCm) for device
memory, ``torch.cuda.current_stream()`` for the stream.  It raises
``ImportError`` if the library has not been built; there is no fallback.
"""
from __future__ import annotations

from ._native import (Batch, CGPError, Guess, Mesh, SolverOpts, StepOpts, abi_version, lib,  # noqa: F401
                      library_path)

__all__ = ["Mesh", "Guess", "Batch", "SolverOpts", "StepOpts", "CGPError", "abi_version", "lib", "library_path"]
