"""Helpers for the GPU parity tests: seeded problems handed identically to the
oracle and to the HIP library."""
import numpy as np
import pytest

import synth
from oracle import Problem


def gpu_ready():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def small_problem(N=96, P=8, tile=32, n_ol=4, ppw=10.0, seed=0, medium="random"):
    """Seeded random-velocity problem with several boxes of uneven shapes."""
    Ng = N + 2 * P
    if medium == "random":
        vel = synth.random_medium(N, P, corr_len_h=6.0, seed=seed)
    else:
        vel = synth.constant_medium(N, P)
    omega = 2 * np.pi * 0.8 * N / ppw
    return Problem(Nx=N, Ny=N, P=P, h=1.0 / N, omega=omega, k_ref=omega, velocity=vel,
                   tile=tile, n_ol=n_ol)


def lib_problem(prob, precision, factor_format=0):
    from paper_1508_02897_amd.solver import make_problem
    return make_problem(prob.Nx, prob.Ny, prob.P, prob.tile or prob.Nx, prob.n_ol, prob.h,
                        prob.omega, prob.k_ref, prob.s0, prob.power, precision, factor_format)


def rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# Complex64 parity bars, per box (max-entry error over a box relative to the
# box's largest value): complex64 rounding of the factors and sweeps (unit
# roundoff 6e-8) amplified by the local condition numbers.  Each is about 3x
# the largest error measured on MI355X for its class of cases:
# line factor on the small layouts (96^2 - 384^2, boxes 52 - 176 wide):
# measured <= 9.9e-6
C64_BOX_BAR = 3e-5
# line factor on the 4096^2 layout's local solves and on 270-wide boxes
# (overlap 50, layer 30): measured <= 2.8e-5
C64_BOX_BAR_WIDE = 1e-4
# nested-dissection local solver (complex128 fronts, complex64 vectors, a
# different elimination order): measured <= 6.1e-5
ND_BOX_BAR = 2e-4


def max_rel(a, b):
    """max |a - b| / max |b|: the worst single entry, relative to the largest
    reference magnitude of the same region."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def box_max_errors(z, ref, prob):
    """For every overlapping box of the decomposition (Sec. 2: tile, overlap
    and the box's own layer), max |z - ref| over the box's nodes relative to
    max |ref| there.  Boxes cover every node, so an error confined to one
    corner box, one layer strip or one edge shows in that box's figure."""
    from oracle.geometry import boxes
    out = []
    for b in boxes(prob):
        (bx0, bx1), (by0, by1) = b["bx"], b["by"]
        out.append(max_rel(z[by0:by1, bx0:bx1], ref[by0:by1, bx0:bx1]))
    return np.array(out)
