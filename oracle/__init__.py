"""FP64 CPU oracle for the one-step overlapping DDM preconditioner (Leng & Ju).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path (the HIP library
and its Python binding) never calls it.  It is a plain, slow, obviously
correct NumPy/SciPy implementation in complex128 of:

* the PML-truncated, 5-point discretised Helmholtz operator (Sec. 2, eq. pml;
  Sec. 3 first paragraph: second-order finite differences)  -> operator.py
* the tile / overlapping-box geometry (Sec. 2, definition of the
  non-overlapping subdomains and of their overlapping extensions) -> geometry.py
* the exact discrete solution by direct solves                  -> direct.py
* the one-step preconditioner (Sec. 2, eq. ddm0 and eq. pc)       -> ddm.py
* restarted right-preconditioned GMRES (Sec. 3)                 -> gmres.py
* the same preconditioner with its local solves in worker processes
  (bitwise equal to ddm.py's)                                    -> pool.py

It shares no code with the GPU path.  Inputs come from the `synth` package.
Every function is pinned by a CPU test against something other than itself
(closed forms, brute force, an independent algorithm); see tests/test_oracle_*.
"""
from .problem import Problem
from . import pml, operator, geometry, direct, ddm, gmres, pool

__all__ = ["Problem", "pml", "operator", "geometry", "direct", "ddm", "gmres", "pool"]
