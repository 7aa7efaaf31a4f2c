"""Pins of the exact discrete solution u* = M^-1 b (three direct routes, one
separable closed form, the free-space Green's function and the PML sign)."""
import numpy as np
import pytest
from scipy.special import hankel1

import synth
from oracle import Problem, direct, operator, pml


def _prob(N, P, vel="random", omega=2 * np.pi * 3.0, seed=0, s0=20.0):
    Ng = N + 2 * P
    if vel == "random":
        rng = np.random.default_rng(seed)
        vel = 1.0 + 0.3 * rng.random((Ng, Ng))
    elif vel == "const":
        vel = np.ones((Ng, Ng))
    return Problem(Nx=N, Ny=N, P=P, h=1.0 / N, omega=omega, k_ref=omega, velocity=vel, s0=s0)


def test_dense_banded_sparse_agree():
    prob = _prob(12, 4)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((20, 20)) + 1j * rng.standard_normal((20, 20))
    ud = direct.dense_solve(prob, f)
    ub = direct.banded_solve(prob, f)
    us = direct.sparse_solve(prob, f)
    n = np.linalg.norm(ud)
    assert np.linalg.norm(ub - ud) <= 1e-12 * n
    assert np.linalg.norm(us - ud) <= 1e-12 * n
    # the solution really solves the brute-force dense system
    M = operator.global_matrix(prob).toarray()
    assert np.linalg.norm(M @ ud.ravel() - f.ravel()) <= 1e-12 * np.linalg.norm(M) * n
    # nonsingular with the layer: smallest singular value well above rounding
    s = np.linalg.svd(M, compute_uv=False)
    assert s[-1] / s[0] > 1e-8


def test_fast_diagonalisation_constant_medium():
    prob = _prob(32, 8, vel="const", omega=2 * np.pi * 4.0)
    f = synth.gaussian_rhs(32, 8, [[0.4, 0.55]], width=2.0 / 32)
    us = direct.sparse_solve(prob, f)
    uf = direct.fast_diag_solve(prob, f)
    assert np.linalg.norm(uf - us) <= 1e-9 * np.linalg.norm(us)


def _green_error(N, k, w, P):
    prob = _prob(N, P, vel="const", omega=k)
    f = synth.gaussian_rhs(N, P, [[0.5, 0.5]], width=w)
    u = direct.sparse_solve(prob, f)
    x = pml.node_x(np.arange(N + 2 * P), P, 1.0 / N)
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X - 0.5, Y - 0.5)
    # Delta u + k^2 u = f with f a unit-mass Gaussian: u -> -(i/4) H0(kr) exp(-k^2 w^2 / 2)
    exact = -0.25j * hankel1(0, k * np.maximum(r, 1e-12)) * np.exp(-0.5 * (k * w) ** 2)
    mask = (r > 0.25) & (r < 0.45)
    return np.linalg.norm((u - exact)[mask]) / np.linalg.norm(exact[mask])


def test_greens_function_second_order():
    """The discrete solution converges to the free-space Green's function at
    second order in h (fixed k, fixed physical source width and layer width)."""
    k, w = 2 * np.pi * 3.0, 0.035
    e = [_green_error(N, k, w, N // 4) for N in (64, 128, 256)]
    orders = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[-1] < 0.01
    assert all(1.7 <= o <= 2.3 for o in orders), (e, orders)


def test_pml_sign_selects_outgoing_wave():
    """With a = 1 + i sigma/k_ref the interior field is the outgoing wave
    -(i/4) H0^(1)(kr) of the Sommerfeld condition; the opposite sign of the
    stretch does not produce it.  The field also decays across the layer, and
    the reflection falls as the layer thickens."""
    N, P = 128, 32
    k, w = 2 * np.pi * 6.0, 0.03
    x = pml.node_x(np.arange(N + 2 * P), P, 1.0 / N)
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X - 0.5, Y - 0.5)
    exact = -0.25j * hankel1(0, k * np.maximum(r, 1e-12)) * np.exp(-0.5 * (k * w) ** 2)
    mask = (r > 0.25) & (r < 0.45)
    f = synth.gaussian_rhs(N, P, [[0.5, 0.5]], width=w)

    def err(s0):
        u = direct.sparse_solve(_prob(N, P, vel="const", omega=k, s0=s0), f)
        return np.linalg.norm((u - exact)[mask]) / np.linalg.norm(exact[mask]), u
    e_plus, u = err(20.0)
    e_minus, _ = err(-20.0)
    assert e_plus < 0.05 and e_minus > 0.5
    mid = P + N // 2
    assert np.abs(u[mid, 0]) < 1e-3 * np.abs(u[mid, P])

    def interior(P):
        ff = synth.gaussian_rhs(64, P, [[0.5, 0.5]], width=2.0 / 64)
        return direct.sparse_solve(_prob(64, P, vel="const", omega=k), ff)[P:P + 64, P:P + 64]
    ref = interior(96)
    e8, e16, e32 = (np.linalg.norm(interior(p) - ref) / np.linalg.norm(ref) for p in (8, 16, 32))
    assert e32 < e16 < e8 < 0.05
