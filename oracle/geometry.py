"""Tiles and overlapping boxes (Sec. 2, definition of the non-overlapping
subdomains, their overlapping extensions by lo + l_pml, and Fig. 1).

Index ranges are in global node indices, half-open.  Along one axis with
N interior nodes, P PML cells per side, tile side n and Nb = N/n tiles:

* tile i covers [P + i n, P + (i+1) n); the first tile also takes the global
  PML strip [0, P) and the last tile the strip [P + N, N + 2P), so the tiles
  partition every node of the truncated grid (reading: the residual inside the
  global PML must reach some local problem, otherwise the preconditioner has a
  null space there).
* box i is the tile's physical interval widened by the overlap lo = n_ol*h on
  interior sides, then by the layer thickness l_pml = P*h on every side.  Its
  physical interval is [a_i, b_i] with a_0 = 0, a_i = (i n - n_ol) h, b_last = N h,
  b_i = ((i+1) n + n_ol) h, and its nodes are those within P*h of [a_i, b_i]:
  start 0 (i = 0) or i n - n_ol, end N + 2P (last) or (i+1) n + n_ol + 2P.
"""
import numpy as np


def tile_range(i, nb, n, P):
    N = nb * n
    lo = 0 if i == 0 else P + i * n
    hi = N + 2 * P if i == nb - 1 else P + (i + 1) * n
    return lo, hi


def box_range(i, nb, n, n_ol, P):
    N = nb * n
    lo = 0 if i == 0 else i * n - n_ol
    hi = N + 2 * P if i == nb - 1 else (i + 1) * n + n_ol + 2 * P
    return lo, hi


def box_physical(i, nb, n, n_ol, h):
    N = nb * n
    a = 0.0 if i == 0 else (i * n - n_ol) * h
    b = N * h if i == nb - 1 else ((i + 1) * n + n_ol) * h
    return a, b


def boxes(prob):
    """List of dicts, lexicographic (iy outer, ix inner)."""
    out = []
    nbx, nby = prob.nbx, prob.nby
    nx = prob.tile if prob.tile else prob.Nx
    ny = prob.tile if prob.tile else prob.Ny
    for iy in range(nby):
        for ix in range(nbx):
            bx = box_range(ix, nbx, nx, prob.n_ol, prob.P)
            by = box_range(iy, nby, ny, prob.n_ol, prob.P)
            tx = tile_range(ix, nbx, nx, prob.P)
            ty = tile_range(iy, nby, ny, prob.P)
            px = box_physical(ix, nbx, nx, prob.n_ol, prob.h)
            py = box_physical(iy, nby, ny, prob.n_ol, prob.h)
            out.append(dict(ix=ix, iy=iy, bx=bx, by=by, tx=tx, ty=ty, px=px, py=py))
    return out
