"""Right-hand sides: superposed normalised Gaussians on interior nodes.

f(x) = sum_s (2*pi*w^2)^-1 * exp(-|x - x_s|^2 / (2 w^2)), width w = 2h, sampled
at interior nodes only (zero in the PML strips).  Centres are drawn uniformly
in [20h, 1-20h]^2 from numpy's default_rng(seed).
"""
import numpy as np
from .media import node_coords


def gaussian_centers(N: int, n_sources: int, seed: int) -> np.ndarray:
    h = 1.0 / N
    rng = np.random.default_rng(seed)
    return rng.uniform(20.0 * h, 1.0 - 20.0 * h, size=(n_sources, 2))


def gaussian_rhs(N: int, P: int, centers, width=None) -> np.ndarray:
    h = 1.0 / N
    w = 2.0 * h if width is None else float(width)
    x = node_coords(N, P)
    Ng = x.size
    f = np.zeros((Ng, Ng), dtype=np.complex128)
    inner = slice(P, P + N)
    xi = x[inner]
    for cx, cy in np.atleast_2d(centers):
        gx = np.exp(-((xi - cx) ** 2) / (2.0 * w * w))
        gy = np.exp(-((xi - cy) ** 2) / (2.0 * w * w))
        f[inner, inner] += np.outer(gy, gx) / (2.0 * np.pi * w * w)
    return f


def rhs_for(w, rhs_index: int = 0) -> np.ndarray:
    """RHS number rhs_index of a Workload: one set of n_sources Gaussians.

    Right-hand side r uses seed source_seed + r.
    """
    c = gaussian_centers(w.N, w.n_sources, w.source_seed + rhs_index)
    return gaussian_rhs(w.N, w.P, c)
