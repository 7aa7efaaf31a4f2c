"""Velocity models sampled at the grid nodes (PML strips included).

* constant: c = c0 everywhere.
* random:   c = 1 + 0.2*g, g a Gaussian random field: white N(0,1) noise on the
            Ng x Ng node grid from numpy's default_rng(seed), circularly
            convolved (FFT) with a Gaussian kernel of standard deviation
            ell/sqrt(2) per axis (covariance proportional to exp(-r^2/(2 ell^2))),
            rescaled to unit empirical standard deviation, clipped to [-1, 1].
* layered:  three layers with c = 1.0 / 1.5 / 2.0 from bottom (y small) to top,
            separated by interfaces y_m(x) = Y_m + 30h*sin(2*pi*q_m*x + phi_m),
            Y = (1/3, 2/3), q_m in {1,2,3} and phi_m in [0, 2*pi) drawn from
            default_rng(seed); the same formula extends into the PML.
"""
import numpy as np


def node_coords(N: int, P: int) -> np.ndarray:
    """Coordinates of the Ng = N + 2P nodes along one axis: (g - P + 1/2)/N."""
    g = np.arange(N + 2 * P, dtype=np.float64)
    return (g - P + 0.5) / N


def constant_medium(N: int, P: int, c0: float = 1.0) -> np.ndarray:
    Ng = N + 2 * P
    return np.full((Ng, Ng), float(c0), dtype=np.float64)


def random_medium(N: int, P: int, corr_len_h: float, seed: int) -> np.ndarray:
    Ng = N + 2 * P
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((Ng, Ng))
    ell = corr_len_h  # in grid cells
    s = ell / np.sqrt(2.0)
    f = np.fft.fftfreq(Ng)  # cycles per cell
    # Fourier transform of a unit-mass Gaussian of std s (cells)
    kern = np.exp(-2.0 * (np.pi * f * s) ** 2)
    g = np.fft.ifft2(np.fft.fft2(white) * kern[:, None] * kern[None, :]).real
    g = g / g.std()
    g = np.clip(g, -1.0, 1.0)
    return 1.0 + 0.2 * g


def layered_medium(N: int, P: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    h = 1.0 / N
    x = node_coords(N, P)
    y = node_coords(N, P)
    q = rng.integers(1, 4, size=2)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=2)
    Y = (1.0 / 3.0, 2.0 / 3.0)
    c = np.full((x.size, x.size), 1.0)
    for m, cval in enumerate((1.5, 2.0)):
        ym = Y[m] + 30.0 * h * np.sin(2.0 * np.pi * q[m] * x + phi[m])  # per column x
        above = y[:, None] > ym[None, :]
        c = np.where(above, cval, c)
    return c


def medium_for(w) -> np.ndarray:
    """Velocity array (Ng, Ng) for a Workload record."""
    if w.medium == "constant":
        return constant_medium(w.N, w.P, 1.0)
    if w.medium == "random":
        return random_medium(w.N, w.P, w.corr_len_h, w.medium_seed)
    if w.medium == "layered":
        return layered_medium(w.N, w.P, w.medium_seed)
    raise ValueError(w.medium)
