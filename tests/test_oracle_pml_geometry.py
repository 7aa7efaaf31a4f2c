"""Pins of the PML stretch tables and of the tile/box geometry (Sec. 2)."""
import numpy as np
import pytest

import synth
from oracle import Problem, pml, geometry


def _prob(N=128, P=16, tile=64, n_ol=8):
    return Problem(Nx=N, Ny=N, P=P, h=1.0 / N, omega=2 * np.pi * 12.8, k_ref=2 * np.pi * 12.8,
                   velocity=np.ones((N + 2 * P, N + 2 * P)), tile=tile, n_ol=n_ol)


def test_stretch_closed_form():
    """a = 1 on every interior node and on the two interface flux points,
    a = 1 + 20i at the outermost flux point, quadratic in between."""
    N, P = 128, 16
    h = 1.0 / N
    a, ah = pml.axis_tables(0, N + 2 * P, P, h, 0.0, 1.0, 20.0, 2)
    assert np.all(a[P:P + N] == 1.0)
    assert ah[P] == 1.0 and ah[P + N] == 1.0          # flux points x = 0 and x = 1
    assert ah[0] == 1 + 20j and ah[-1] == 1 + 20j      # x = -P h and 1 + P h
    # node 0 lies (P - 1/2) h outside: 20 * (15.5/16)^2 = 18.76953125
    assert a[0] == pytest.approx(1 + 18.76953125j, abs=1e-13)
    assert a[-1] == pytest.approx(1 + 18.76953125j, abs=1e-13)
    # flux point 8 lies 8h outside: 20 * (8/16)^2 = 5
    assert ah[8] == pytest.approx(1 + 5j, abs=1e-13)
    assert np.all(np.diff(a[:P].imag) < 0) and np.all(np.diff(a[P + N:].imag) > 0)


def test_c1_boxes_and_tiles():
    prob = _prob()
    bs = geometry.boxes(prob)
    assert len(bs) == 4
    assert [b["bx"] for b in bs[:2]] == [(0, 104), (56, 160)]
    assert [b["tx"] for b in bs[:2]] == [(0, 80), (80, 160)]
    assert bs[0]["px"] == (0.0, (64 + 8) / 128) and bs[1]["px"] == ((64 - 8) / 128, 1.0)


@pytest.mark.parametrize("nb", [1, 2, 3, 8])
def test_tiles_partition_and_cover(nb):
    n, P, n_ol = 32, 8, 4
    N = nb * n
    Ng = N + 2 * P
    prob = _prob(N=N, P=P, tile=n, n_ol=n_ol)
    tile_count = np.zeros((Ng, Ng), int)
    box_count = np.zeros((Ng, Ng), int)
    for b in geometry.boxes(prob):
        (tx0, tx1), (ty0, ty1) = b["tx"], b["ty"]
        (bx0, bx1), (by0, by1) = b["bx"], b["by"]
        tile_count[ty0:ty1, tx0:tx1] += 1
        box_count[by0:by1, bx0:bx1] += 1
        # tile inside its box, box nodes exactly those within P h of the physical interval
        assert bx0 <= tx0 and tx1 <= bx1 and by0 <= ty0 and ty1 <= by1
        x = pml.node_x(np.arange(Ng), P, 1.0 / N)
        inside = (x >= b["px"][0] - P / N - 1e-12) & (x <= b["px"][1] + P / N + 1e-12)
        assert np.flatnonzero(inside)[0] == bx0 and np.flatnonzero(inside)[-1] == bx1 - 1
    assert np.all(tile_count == 1)
    assert box_count.max() <= 4 and box_count.min() >= 1
    if nb == 1:
        assert geometry.boxes(prob)[0]["bx"] == (0, Ng)


def test_box_sides_for_128_tiles():
    for name in ("c2_1024", "c4_4096"):
        w = synth.config(name)
        sides = [geometry.box_range(i, w.nb, w.tile, w.n_ol, w.P) for i in range(w.nb)]
        widths = [b - a for a, b in sides]
        assert widths[0] == widths[-1] == 168 and set(widths[1:-1]) == {176}
