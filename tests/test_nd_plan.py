"""Host logic of the nested-dissection local solver (no GPU): the factor size
the library plans for every box equals the count of the separator tree built
here by the same rule (halve the longer side of a rectangle by a separator
line down to rectangles of at most 16 nodes; a front keeps G (s x s), L
(b x s) and L^T (s x b), complex128, for its s separator nodes and the b nodes
of its rectangle's ring), and the format is refused where it does not apply."""
import numpy as np
import pytest

import synth
from oracle import geometry
from oracle.problem import Problem

LEAF = 16


def _front_entries(mx, my):
    """Sum over fronts of s^2 + 2 b s for one mx x my box."""
    tot = 0
    stack = [(0, my, 0, mx)]
    while stack:
        y0, y1, x0, x1 = stack.pop()
        h, w = y1 - y0, x1 - x0
        if h <= 0 or w <= 0:
            continue
        b = (x1 - x0) * ((y0 > 0) + (y1 < my)) + (y1 - y0) * ((x0 > 0) + (x1 < mx))
        if h * w <= LEAF:
            s = h * w
        elif h >= w:
            m = y0 + h // 2
            s = w
            stack += [(y0, m, x0, x1), (m + 1, y1, x0, x1)]
        else:
            m = x0 + w // 2
            s = h
            stack += [(y0, y1, x0, m), (y0, y1, m + 1, x1)]
        tot += s * s + 2 * b * s
    return tot


def _lib(w, precision, fmt):
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import problem_from_workload
    return H.hddm_setup(problem_from_workload(w, precision, fmt), synth.medium_for(w), 0)


@pytest.mark.parametrize("name", ["c1_128", "c2_1024"])
def test_nd_factor_bytes_match_separator_tree(name):
    from paper_1508_02897_amd import hddm as H
    w = synth.config(name)
    ctx = _lib(w, H.HDDM_MIXED_C64, H.FORMAT_NESTED_DISSECTION)
    fb, wb, _ = H.hddm_query_bytes(ctx, 10)
    H.hddm_destroy(ctx)
    prob = Problem.from_workload(w)
    want = 0
    for bx in geometry.boxes(prob):
        mx = bx["bx"][1] - bx["bx"][0]
        my = bx["by"][1] - bx["by"][0]
        want += (_front_entries(mx, my) + 31) // 32 * 32
    assert fb == want * 16  # complex128 fronts
    # the line factor of the same problem streams more entries per node
    ctx = _lib(w, H.HDDM_MIXED_C64, H.FORMAT_AUTO)
    fb_line, _, _ = H.hddm_query_bytes(ctx, 10)
    H.hddm_destroy(ctx)
    print(name, "nested dissection", fb / 1e6, "MB; line factor", fb_line / 1e6, "MB")


def test_nd_needs_complex64():
    from paper_1508_02897_amd import hddm as H
    with pytest.raises(RuntimeError, match="HDDM_MIXED_C64"):
        _lib(synth.config("c1_128"), H.HDDM_PLAIN_C128, H.FORMAT_NESTED_DISSECTION)


def test_nd_front_entries_small_box():
    """Hand count for a 5 x 4 box: one vertical separator of 4 nodes
    (area 20 > 16, x is the longer side) with two leaves of 2 x 4 and 2 x 4."""
    # leaves: s = 8, ring = the 4 separator nodes -> 64 + 2*4*8 each; root: 16
    assert _front_entries(5, 4) == 2 * (64 + 64) + 16


def _setup_nd(N, P, tile, n_ol):
    import numpy as np
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import make_problem
    om = 2 * np.pi * 0.8 * N / 10
    p = make_problem(N, N, P, tile, n_ol, 1.0 / N, om, om, 20.0, 2, H.HDDM_MIXED_C64,
                     H.FORMAT_NESTED_DISSECTION)
    return H.hddm_setup(p, np.ones((N + 2 * P, N + 2 * P)), 0)


def test_nd_serves_boxes_wider_than_the_line_block_form():
    """Boxes 270 wide (overlap 50, layer 30): beyond the packed line factor
    (256) and its block form (192), within the fronts the solver takes."""
    from paper_1508_02897_amd import hddm as H
    ctx = _setup_nd(320, 30, 160, 50)
    nbx, nby, boxes = H.hddm_geometry(ctx)
    assert int((boxes[:, 1] - boxes[:, 0]).max()) == 270
    wb, kb = H.hddm_query_block_bytes(ctx, 16, 3)
    assert wb > 0 and kb > 0
    H.hddm_destroy(ctx)


def test_nd_rejects_fronts_too_large():
    """Interior boxes 320 wide: a front of 160 separator and 320 ring nodes
    exceeds what the solve kernels stage in LDS; setup refuses with EINVAL."""
    with pytest.raises(RuntimeError, match="too large"):
        _setup_nd(480, 30, 160, 50)
