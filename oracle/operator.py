"""Second-order finite-difference PML operator (Sec. 2, eq. pml; Sec. 3).

The truncated problem J^-1 div(A grad u) + k^2 u = f with A = diag(a2/a1, a1/a2)
and J = a1*a2 is multiplied through by J, giving

    d/dx( (a2/a1) du/dx ) + d/dy( (a1/a2) du/dy ) + k^2 a1 a2 u = J f.

Since a2 depends on y only and a1 on x only this is
a2 * d/dx( a1^-1 du/dx ) + a1 * d/dy( a2^-1 du/dy ) + k^2 a1 a2 u, discretised
on a cell-centred grid with fluxes at half nodes:

    (M u)_p = cE (uE - u) + cW (uW - u) + cN (uN - u) + cS (uS - u) + k^2 a1 a2 u
    cE = a2 / (h^2 a1(x + h/2)),  cW = a2 / (h^2 a1(x - h/2)),
    cN = a1 / (h^2 a2(y + h/2)),  cS = a1 / (h^2 a2(y - h/2)).

Neighbours outside the grid carry u = 0 (homogeneous Dirichlet one node past
the layer).  The matrix is complex symmetric.  Unknown ordering: row-major
(y outer, x fastest), matching the (Ny, Nx) array layout.
"""
import numpy as np
import scipy.sparse as sp


def assemble(ax, hx, ay, hy, k2, h):
    """Sparse M for an mx-by-my block of nodes.

    ax (mx,), hx (mx+1,): stretch at x nodes / x flux points; ay, hy likewise.
    k2 (my, mx): squared wave number at the nodes.
    """
    mx, my = ax.size, ay.size
    assert hx.size == mx + 1 and hy.size == my + 1 and k2.shape == (my, mx)
    inv_h2 = 1.0 / (h * h)
    A1 = ax[None, :]
    A2 = ay[:, None]
    cW = A2 * inv_h2 / hx[None, :-1]
    cE = A2 * inv_h2 / hx[None, 1:]
    cS = A1 * inv_h2 / hy[:-1, None]
    cN = A1 * inv_h2 / hy[1:, None]
    cW = np.broadcast_to(cW, (my, mx)); cE = np.broadcast_to(cE, (my, mx))
    cS = np.broadcast_to(cS, (my, mx)); cN = np.broadcast_to(cN, (my, mx))
    diag = -(cW + cE + cS + cN) + k2 * A1 * A2
    idx = np.arange(mx * my).reshape(my, mx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    # east / west neighbours
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(cE[:, :-1].ravel())
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(cW[:, 1:].ravel())
    # north / south neighbours
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(cN[:-1, :].ravel())
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(cS[1:, :].ravel())
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mx * my, mx * my)).tocsr()
    return M


def global_tables(prob):
    """Stretch tables of the whole truncated domain: the physical region is
    the interior [0, Nx h] x [0, Ny h]."""
    from .pml import axis_tables
    ax, hx = axis_tables(0, prob.Ngx, prob.P, prob.h, 0.0, prob.Nx * prob.h, prob.s0, prob.power)
    ay, hy = axis_tables(0, prob.Ngy, prob.P, prob.h, 0.0, prob.Ny * prob.h, prob.s0, prob.power)
    return ax, hx, ay, hy


def global_matrix(prob):
    ax, hx, ay, hy = global_tables(prob)
    return assemble(ax, hx, ay, hy, prob.k2(), prob.h)


def apply_stencil(u, ax, hx, ay, hy, k2, h):
    """Matrix-free M u on a (my, mx) array: the same definition as assemble()."""
    inv_h2 = 1.0 / (h * h)
    A1 = ax[None, :]
    A2 = ay[:, None]
    up = np.pad(u, 1)
    uc = u
    uE = up[1:-1, 2:]; uW = up[1:-1, :-2]; uN = up[2:, 1:-1]; uS = up[:-2, 1:-1]
    cW = A2 * inv_h2 / hx[None, :-1]
    cE = A2 * inv_h2 / hx[None, 1:]
    cS = A1 * inv_h2 / hy[:-1, None]
    cN = A1 * inv_h2 / hy[1:, None]
    return (cE * (uE - uc) + cW * (uW - uc) + cN * (uN - uc) + cS * (uS - uc)
            + k2 * A1 * A2 * uc)


def matvec(prob, u):
    ax, hx, ay, hy = global_tables(prob)
    return apply_stencil(u, ax, hx, ay, hy, prob.k2(), prob.h)


def stencil_at(prob, u, iy, ix):
    """(M u) at the listed nodes only, each computed from its five neighbours
    (for spot checks on grids too large to assemble)."""
    ax, hx, ay, hy = global_tables(prob)
    inv_h2 = 1.0 / (prob.h * prob.h)
    iy = np.asarray(iy); ix = np.asarray(ix)
    Ny, Nx = u.shape

    def get(j, i):
        ok = (j >= 0) & (j < Ny) & (i >= 0) & (i < Nx)
        out = np.zeros(j.shape, dtype=np.complex128)
        out[ok] = u[j[ok], i[ok]]
        return out
    a1 = ax[ix]; a2 = ay[iy]
    cW = a2 * inv_h2 / hx[ix]; cE = a2 * inv_h2 / hx[ix + 1]
    cS = a1 * inv_h2 / hy[iy]; cN = a1 * inv_h2 / hy[iy + 1]
    uc = u[iy, ix]
    k2 = (prob.omega / prob.velocity[iy, ix]) ** 2
    return (cE * (get(iy, ix + 1) - uc) + cW * (get(iy, ix - 1) - uc)
            + cN * (get(iy + 1, ix) - uc) + cS * (get(iy - 1, ix) - uc)
            + k2 * a1 * a2 * uc)
