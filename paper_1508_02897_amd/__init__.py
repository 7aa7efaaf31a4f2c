"""MI355X (gfx950) library for the one-step overlapping DDM preconditioner of
Leng & Ju for the 2D PML-truncated Helmholtz equation.

`hddm` is the ctypes binding of the C ABI (include/hddm.h); `solver.Solver`
owns torch device buffers for one medium and forwards to the library.
"""
from . import hddm
from .hddm import HddmError, HDDM_PLAIN_C128, HDDM_MIXED_C64

__all__ = ["hddm", "HddmError", "HDDM_PLAIN_C128", "HDDM_MIXED_C64"]
