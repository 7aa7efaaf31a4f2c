"""Uniaxial PML stretch factors (Sec. 2, the stretched coordinates and eq. pml).

The paper stretches each coordinate separately with a damping profile sigma_j
that vanishes inside the physical region and is positive in the layer, and
writes the truncated operator with A = diag(a2/a1, a1/a2), J = a1*a2, where the
stretch factor a_j is left undefined in the printed text.  Reading used here:

    a(t) = 1 + i * sigma(t) / k_ref,   sigma(t) = s0 * k_ref * (d(t) / L)^power,

with d(t) the distance of t outside the physical interval and L the layer
thickness.  The +i sign makes the outgoing wave exp(+i k r) of the Sommerfeld
condition (Sec. 1, eq. helm) decay inside the layer.
"""
import numpy as np


def node_x(g, P, h):
    """Coordinate of node index g (may be a half-integer for flux points)."""
    return (np.asarray(g, dtype=np.float64) - P + 0.5) * h


def stretch(t, lo, hi, L, s0, power=2):
    """a(t) for the physical interval [lo, hi] with layer thickness L."""
    t = np.asarray(t, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(lo - t, t - hi))
    return 1.0 + 1j * s0 * (d / L) ** power


def axis_tables(g0, m, P, h, lo, hi, s0, power=2):
    """Stretch at the m nodes g0..g0+m-1 and at the m+1 flux points between
    and around them (node g0+i has flux points g0+i-1/2 and g0+i+1/2)."""
    L = P * h
    nodes = node_x(np.arange(g0, g0 + m), P, h)
    halves = node_x(np.arange(g0, g0 + m + 1) - 0.5, P, h)
    return stretch(nodes, lo, hi, L, s0, power), stretch(halves, lo, hi, L, s0, power)
