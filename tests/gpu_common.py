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
