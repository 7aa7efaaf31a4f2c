"""The one-step overlapping DDM preconditioner (Sec. 2, eq. ddm0 and eq. pc).

For every overlapping box Omega_ij the local PML problem (eq. pmlij) is set up
with the box's own layer: the stretch uses the distance outside the box's
physical interval [a_i, b_i] x [a_j, b_j] (tile plus overlap), the squared wave
number is the global medium at the same nodes (also inside the local layer),
and the box edge carries u = 0 one node past its layer.  The preconditioner
applied to a global residual r is

    z = sum_ij E_ij  M_ij^-1  R~_ij r,

where R~_ij keeps r on the tile's nodes and zero elsewhere in the box (the
source restricted to the non-overlapping subdomain, eq. ddm0) and E_ij adds
the local solution back over the whole box, layer included (eq. pc).  By
default the smoothing function of the Remark after eq. pc is omitted, as in
the paper's experiments; smooth=True multiplies each local solution by its
box's beta_ij before the sum (see `smoothing`).

Local solves use SuperLU on the assembled local matrix, a different algorithm
from the block-tridiagonal factorisation of the GPU path by design.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .geometry import boxes
from .operator import assemble
from .pml import axis_tables


def local_tables(prob, box):
    bx0, bx1 = box["bx"]; by0, by1 = box["by"]
    ax, hx = axis_tables(bx0, bx1 - bx0, prob.P, prob.h, box["px"][0], box["px"][1], prob.s0, prob.power)
    ay, hy = axis_tables(by0, by1 - by0, prob.P, prob.h, box["py"][0], box["py"][1], prob.s0, prob.power)
    # the squared wave number on the box's nodes only (the same elementwise
    # (omega / c)^2 as Problem.k2, without forming it over the whole grid)
    k2 = (prob.omega / prob.velocity[by0:by1, bx0:bx1]) ** 2
    return ax, hx, ay, hy, k2


def local_matrix(prob, box):
    ax, hx, ay, hy, k2 = local_tables(prob, box)
    return assemble(ax, hx, ay, hy, k2, prob.h)


def restrict(r, box):
    """Local source: r on the tile's nodes, zero in the overlap and layer."""
    bx0, bx1 = box["bx"]; by0, by1 = box["by"]
    tx0, tx1 = box["tx"]; ty0, ty1 = box["ty"]
    b = np.zeros((by1 - by0, bx1 - bx0), dtype=np.complex128)
    b[ty0 - by0:ty1 - by0, tx0 - bx0:tx1 - bx0] = r[ty0:ty1, tx0:tx1]
    return b


def ramp_weights(t0, t1, b0, b1):
    """One axis of beta_ij (Sec. 2, Remark after eq. pc): 1 on the tile's nodes
    [t0, t1), falling to 0 at the box edges b0 <= t0, b1 >= t1.  The paper only
    asks for beta in C^2, equal to 1 on the tile and 0 outside the box; the
    reading used here: across each side's strip (overlap and layer) of width
    L, at the cell-centred node a distance (d + 1/2) cells past the tile edge,
    beta = 1 - S((d + 1/2) / L) with S(s) = 10 s^3 - 15 s^4 + 6 s^5, the quintic
    whose first and second derivatives vanish at s = 0 and s = 1."""
    n = b1 - b0
    w = np.ones(n)
    g = np.arange(b0, b1)

    def drop(s):
        return 1.0 - s ** 3 * (10.0 - 15.0 * s + 6.0 * s ** 2)

    left = g < t0
    if left.any():
        w[left] = drop((t0 - g[left] - 0.5) / (t0 - b0))
    right = g >= t1
    if right.any():
        w[right] = drop((g[right] - t1 + 0.5) / (b1 - t1))
    return w


def smoothing(box):
    """beta_ij on the box's nodes: the product of the two axes' ramps."""
    wx = ramp_weights(box["tx"][0], box["tx"][1], box["bx"][0], box["bx"][1])
    wy = ramp_weights(box["ty"][0], box["ty"][1], box["by"][0], box["by"][1])
    return np.outer(wy, wx)


# SuperLU options of a low-fill factorisation for the large workloads: minimum
# degree on the symmetric pattern of A + A^T with a small diagonal pivoting
# threshold (the local matrices are complex symmetric).  About half the fill of
# the default column ordering on a 176-wide box; the local solve is the same
# exact solve, only rounded differently.
LOW_FILL = dict(permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.01,
                options=dict(SymmetricMode=True))


def local_factor(prob, box, splu_options=None):
    """SuperLU factorisation of the box's local matrix M_ij."""
    return spla.splu(local_matrix(prob, box).tocsc(), **(splu_options or {}))


class OneStepDDM:
    def __init__(self, prob, boxes_subset=None, smooth=False, splu_options=None):
        self.prob = prob
        self.smooth = smooth
        self.boxes = boxes(prob)
        self.ids = range(len(self.boxes)) if boxes_subset is None else list(boxes_subset)
        self.lu = {}
        for i in self.ids:
            self.lu[i] = local_factor(prob, self.boxes[i], splu_options)

    def local_solve(self, i, r):
        box = self.boxes[i]
        b = restrict(r, box)
        return self.lu[i].solve(b.ravel()).reshape(b.shape)

    def apply(self, r):
        z = np.zeros_like(r, dtype=np.complex128)
        for i in self.ids:
            box = self.boxes[i]
            u = self.local_solve(i, r)
            if self.smooth:
                u = smoothing(box) * u
            bx0, bx1 = box["bx"]; by0, by1 = box["by"]
            z[by0:by1, bx0:bx1] += u
        return z


def neighbours(prob, i):
    """N_ij (Sec. 2): the up to 8 boxes (i', j') with |i' - i| <= 1,
    |j' - j| <= 1, (i', j') != (i, j); boxes are numbered i = iy * nbx + ix."""
    iy, ix = divmod(i, prob.nbx)
    out = []
    for jy in (iy - 1, iy, iy + 1):
        for jx in (ix - 1, ix, ix + 1):
            if (jy, jx) != (iy, ix) and 0 <= jy < prob.nby and 0 <= jx < prob.nbx:
                out.append(jy * prob.nbx + jx)
    return out


def multistep(prob, f, steps, tol=None):
    """The iterative overlapping DDM of eq. ddm0 / eq. ddms / eq. sum, step by
    step as the paper writes it: step 0 solves every box with f restricted to
    its tile; step s+1 solves box (i, j) with the source
        - sum over (i', j') in N_ij of  L(u^s_{i'j'})  restricted to the tile,
    each neighbour's local solution extended by zero outside its box and L
    taken as the discrete global operator M (the local problems are solved in
    the same form, M_ij u = b_ij, Sec. 2 with the reading of eq. pml x J); the
    result is the sum of all local solutions of all steps.  Stops after
    `steps` steps, or earlier once the global residual |f - M u| / |f| of the
    running sum is <= tol.  Returns (u, relres after each step)."""
    from .operator import matvec
    P = OneStepDDM(prob)
    bx = P.boxes
    nb = np.linalg.norm(f)
    ext = {}

    def extend(i, u):
        e = np.zeros(f.shape, dtype=np.complex128)
        (bx0, bx1), (by0, by1) = bx[i]["bx"], bx[i]["by"]
        e[by0:by1, bx0:bx1] = u
        return e

    u_sum = np.zeros(f.shape, dtype=np.complex128)
    for i in P.ids:  # step 0
        ext[i] = extend(i, P.local_solve(i, f))
        u_sum += ext[i]
    hist = [np.linalg.norm(f - matvec(prob, u_sum)) / nb]
    for s in range(1, steps):
        if tol is not None and hist[-1] <= tol:
            break
        Lu = {i: matvec(prob, ext[i]) for i in P.ids}
        new = {}
        for i in P.ids:
            src = np.zeros(f.shape, dtype=np.complex128)
            for j in neighbours(prob, i):
                src -= Lu[j]
            new[i] = extend(i, P.local_solve(i, src))  # local_solve keeps src on the tile
        ext = new
        for i in P.ids:
            u_sum += ext[i]
        hist.append(np.linalg.norm(f - matvec(prob, u_sum)) / nb)
    return u_sum, hist
