"""Exact discrete solution u* = M^-1 b by direct methods (the plain
definition of what the preconditioned iteration converges to).

Three independent routes, used against each other in the tests:
* dense LU (numpy.linalg.solve) on tiny grids,
* banded LU (scipy.linalg.solve_banded, bandwidth Ngx) on small grids,
* sparse LU (scipy SuperLU) on larger grids,
plus, for a constant medium, fast diagonalisation of the separable operator
(eigen-decomposition of the two 1D stretched second-difference operators),
which does not assemble the 2D matrix at all.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import global_matrix, global_tables


def dense_solve(prob, f):
    M = global_matrix(prob).toarray()
    return np.linalg.solve(M, f.ravel()).reshape(f.shape)


def banded_solve(prob, f):
    M = global_matrix(prob).tocsr()
    bw = prob.Ngx
    n = M.shape[0]
    ab = np.zeros((2 * bw + 1, n), dtype=np.complex128)
    coo = M.tocoo()
    ab[bw + coo.row - coo.col, coo.col] = coo.data
    return sla.solve_banded((bw, bw), ab, f.ravel()).reshape(f.shape)


def sparse_solve(prob, f):
    M = global_matrix(prob).tocsc()
    lu = spla.splu(M)
    return lu.solve(f.ravel()).reshape(f.shape)


def _second_difference(hx, h):
    """1D operator D v = [(v_{i+1}-v_i)/a_{i+1/2} - (v_i-v_{i-1})/a_{i-1/2}] / h^2
    with zero values beyond both ends (dense, small)."""
    m = hx.size - 1
    w = 1.0 / (h * h * hx)
    D = np.diag(-(w[:-1] + w[1:])) + np.diag(w[1:-1], 1) + np.diag(w[1:-1], -1)
    return D.astype(np.complex128)


def fast_diag_solve(prob, f):
    """Constant medium only: a2*Dx + a1*Dy + k^2 a1 a2 = (A2 x A1)(Lx + Ly + k^2)
    with Lx = A1^-1 Dx, so u = (Vy x Vx) diag(1/(ly + lx + k^2)) (Vy x Vx)^-1 (A2 x A1)^-1 f."""
    k2 = prob.k2()
    assert np.allclose(k2, k2.flat[0]), "fast diagonalisation needs a constant medium"
    k2 = k2.flat[0]
    ax, hx, ay, hy = global_tables(prob)
    Lx = _second_difference(hx, prob.h) / ax[:, None]
    Ly = _second_difference(hy, prob.h) / ay[:, None]
    lx, Vx = np.linalg.eig(Lx)
    ly, Vy = np.linalg.eig(Ly)
    g = f / (ay[:, None] * ax[None, :])
    ghat = np.linalg.solve(Vy, np.linalg.solve(Vx, g.T).T)
    uhat = ghat / (ly[:, None] + lx[None, :] + k2)
    return Vy @ uhat @ Vx.T
