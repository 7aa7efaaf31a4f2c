"""Pins of the discrete PML operator (Sec. 2 eq. pml, Sec. 3 second-order FD)."""
import numpy as np
import scipy.sparse as sp

from oracle import Problem, operator, direct, pml


def _prob(N, P, vel=None, omega=2 * np.pi * 4.0, seed=0):
    Ng = N + 2 * P
    if vel == "random":
        rng = np.random.default_rng(seed)
        vel = 1.0 + 0.3 * rng.random((Ng, Ng))
    elif vel is None:
        vel = np.ones((Ng, Ng))
    return Problem(Nx=N, Ny=N, P=P, h=1.0 / N, omega=omega, k_ref=omega, velocity=vel)


def test_complex_symmetric_bitwise():
    prob = _prob(40, 8, "random")
    M = operator.global_matrix(prob)
    D = (M - M.T)
    assert abs(D).max() == 0.0
    # not Hermitian: the layer makes it genuinely complex
    assert abs(M - M.conj().T).max() > 0


def test_kronecker_assembly_agrees():
    """Second construction from 1D operators: M = A2 x D1 + D2 x A1 + diag(k^2 a1 a2)."""
    prob = _prob(24, 6, "random")
    ax, hx, ay, hy = operator.global_tables(prob)
    h = prob.h

    def d1(half):
        w = 1.0 / (h * h * half)
        return sp.diags([-(w[:-1] + w[1:]), w[1:-1], w[1:-1]], [0, 1, -1])
    K = sp.kron(sp.diags(ay), d1(hx)) + sp.kron(d1(hy), sp.diags(ax)) \
        + sp.diags((prob.k2() * np.outer(ay, ax)).ravel())
    M = operator.global_matrix(prob)
    assert abs(M - K).max() <= 1e-14 * abs(M).max()
    # matrix-free stencil and spot evaluation agree with the matrix
    rng = np.random.default_rng(3)
    u = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    Mu = (M @ u.ravel()).reshape(u.shape)
    assert np.abs(operator.matvec(prob, u) - Mu).max() <= 1e-13 * np.abs(Mu).max()
    iy = np.array([0, 5, 17, prob.Ngy - 1]); ix = np.array([prob.Ngx - 1, 0, 9, 3])
    assert np.abs(operator.stencil_at(prob, u, iy, ix) - Mu[iy, ix]).max() <= 1e-13 * np.abs(Mu).max()


def test_interior_rows_annihilate_discrete_plane_wave():
    """(4/h^2) sin^2(kappa h/2) = k^2 makes exp(i kappa x) an exact null vector of
    the interior 5-point rows (constant medium, a = 1 there)."""
    N, P = 64, 8
    prob = _prob(N, P, omega=2 * np.pi * 6.0)
    h = prob.h
    k = prob.omega
    kappa = 2.0 / h * np.arcsin(k * h / 2.0)
    x = pml.node_x(np.arange(N + 2 * P), P, h)
    for direction in ("x", "y", "diag"):
        if direction == "x":
            u = np.exp(1j * kappa * x)[None, :] * np.ones((N + 2 * P, 1))
        elif direction == "y":
            u = np.exp(1j * kappa * x)[:, None] * np.ones((1, N + 2 * P))
        else:
            kd = 2.0 / h * np.arcsin(k * h / 2.0 / np.sqrt(2.0))
            u = np.exp(1j * kd * (x[None, :] + x[:, None]))
        r = operator.matvec(prob, u)
        inner = slice(P + 1, P + N - 1)
        assert np.abs(r[inner, inner]).max() <= 1e-9 * (4 / h ** 2)
        # the layer rows do not annihilate it
        assert np.abs(r[:P, :]).max() > 1e-3 * (4 / h ** 2) or np.abs(r[:, :P]).max() > 1e-3 * (4 / h ** 2)


def test_reciprocity():
    prob = _prob(20, 6, "random", seed=5)
    Ng = prob.Ngx
    a, b = (9, 11), (22, 14)
    ea = np.zeros((Ng, Ng), complex); ea[a] = 1
    eb = np.zeros((Ng, Ng), complex); eb[b] = 1
    ua = direct.sparse_solve(prob, ea)
    ub = direct.sparse_solve(prob, eb)
    assert abs(ua[b] - ub[a]) <= 1e-12 * abs(ua[b])
