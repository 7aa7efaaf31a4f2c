"""Problem record of the oracle: grid, PML, medium, decomposition."""
from dataclasses import dataclass
import numpy as np


@dataclass
class Problem:
    Nx: int                 # interior nodes along x (h = 1/N with N = Nx for the unit square)
    Ny: int
    P: int                  # PML cells per side
    h: float
    omega: float
    k_ref: float
    velocity: np.ndarray    # (Ny + 2P, Nx + 2P) float64
    tile: int = 0           # tile side (0: single tile)
    n_ol: int = 0
    s0: float = 20.0        # sigma0 / k_ref
    power: int = 2

    @property
    def Ngx(self):
        return self.Nx + 2 * self.P

    @property
    def Ngy(self):
        return self.Ny + 2 * self.P

    @property
    def nbx(self):
        return self.Nx // self.tile if self.tile else 1

    @property
    def nby(self):
        return self.Ny // self.tile if self.tile else 1

    def k2(self):
        return (self.omega / self.velocity) ** 2

    @classmethod
    def from_workload(cls, w, velocity=None):
        from synth import medium_for
        vel = medium_for(w) if velocity is None else velocity
        return cls(Nx=w.N, Ny=w.N, P=w.P, h=w.h, omega=w.omega, k_ref=w.k_ref,
                   velocity=vel, tile=w.tile, n_ol=w.n_ol,
                   s0=w.sigma0_over_kref, power=w.pml_power)
