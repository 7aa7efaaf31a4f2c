"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package draws the *inputs* of a Helmholtz solve (velocity models,
right-hand sides, workload parameters) and nothing else: it holds none of the
discretisation, PML, decomposition or Krylov arithmetic.  Both the oracle and
the HIP library receive the arrays it returns.

Layout convention for every grid array: shape (Ngy, Ngx), row-major, x fastest,
covering the whole truncated domain including the PML strips.  Node g along an
axis sits at coordinate (g - P + 1/2) * h with h = 1/N, so nodes P .. P+N-1
cover the unit interval and P nodes on each side lie in the PML.
"""
from .configs import CONFIGS, config, Workload
from .media import node_coords, constant_medium, random_medium, layered_medium, medium_for
from .sources import gaussian_centers, gaussian_rhs, rhs_for

__all__ = [
    "CONFIGS", "config", "Workload", "node_coords", "constant_medium",
    "random_medium", "layered_medium", "medium_for", "gaussian_centers",
    "gaussian_rhs", "rhs_for",
]
