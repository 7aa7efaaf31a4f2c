"""Workload records for the benchmark and parity configurations.

Each record fixes the grid (N interior nodes per side, P PML cells), the
decomposition (tile side n, overlap n_ol), the angular frequency omega, the
medium generator and the sources.  omega follows the points-per-wavelength
rule omega = 2*pi*c_min*N/ppw with the generator's nominal minimum velocity
c_min, and the PML reference wave number is k_ref = omega / 1.0.
"""
from dataclasses import dataclass, field
import math


@dataclass(frozen=True)
class Workload:
    name: str
    N: int                  # interior nodes per side (square unit domain)
    P: int                  # PML cells on each side
    tile: int               # tile side n (N % tile == 0)
    n_ol: int               # overlap cells on interior sides
    ppw: float              # points per wavelength at c_min
    c_min: float            # nominal minimum velocity of the medium
    medium: str             # "constant" | "random" | "layered"
    medium_seed: int = 0
    corr_len_h: float = 20.0   # random medium correlation length in units of h
    n_sources: int = 1
    source_seed: int = 1
    n_rhs: int = 1
    restart: int = 50
    tol: float = 1e-8
    sigma0_over_kref: float = 20.0
    pml_power: int = 2

    @property
    def Ng(self) -> int:
        return self.N + 2 * self.P

    @property
    def h(self) -> float:
        return 1.0 / self.N

    @property
    def nb(self) -> int:
        return self.N // self.tile

    @property
    def omega(self) -> float:
        return 2.0 * math.pi * self.c_min * self.N / self.ppw

    @property
    def k_ref(self) -> float:
        return self.omega / 1.0


CONFIGS = {
    # 128^2 interior, 2x2 tiles of 64, constant c=1, 10 ppw (k = 2*pi*12.8)
    "c1_128": Workload("c1_128", N=128, P=16, tile=64, n_ol=8, ppw=10.0, c_min=1.0,
                       medium="constant", n_sources=1, source_seed=1),
    # 1024^2, 8x8 tiles of 128, random medium (corr 20h), 4 superposed sources
    "c2_1024": Workload("c2_1024", N=1024, P=16, tile=128, n_ol=8, ppw=10.0, c_min=0.8,
                        medium="random", medium_seed=2, corr_len_h=20.0,
                        n_sources=4, source_seed=2),
    # 2048^2, 16x16 tiles of 128, 3-layer medium, 12 ppw
    "c3_2048": Workload("c3_2048", N=2048, P=16, tile=128, n_ol=8, ppw=12.0, c_min=1.0,
                        medium="layered", medium_seed=3, n_sources=1, source_seed=3),
    # 4096^2, 32x32 tiles of 128, random medium (corr 40h), 16 right-hand sides
    "c4_4096": Workload("c4_4096", N=4096, P=16, tile=128, n_ol=8, ppw=10.0, c_min=0.8,
                        medium="random", medium_seed=4, corr_len_h=40.0,
                        n_sources=1, source_seed=4000, n_rhs=16),
}


def config(name: str) -> Workload:
    return CONFIGS[name]
