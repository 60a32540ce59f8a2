"""MI355X (gfx950) matrix-free SIPG operators: Python binding of libsipg.

A thin ctypes layer over the C ABI in include/sipg.h: it marshals arguments,
hands torch device pointers and the current HIP stream to the library, and
allocates the plan's workspace as a torch tensor.  Every step of the
operator, diagonal and solve runs in the library's HIP kernels; there is no
Python or CPU fallback, and importing this package fails if the library has
not been built (python -m paper_2506_14424_amd.build).
"""
from __future__ import annotations

from ._ffi import (LIB_PATH, SipgError, lib, PART_CELL, PART_INTERIOR, PART_BOUNDARY,
                   PART_ALL)
from .operator import Operator, SolveOptions
from .splitting import SplitOptions, SplitStep

__all__ = ["Operator", "SolveOptions", "SplitStep", "SplitOptions", "SipgError", "lib", "LIB_PATH",
           "PART_CELL", "PART_INTERIOR", "PART_BOUNDARY", "PART_ALL"]
