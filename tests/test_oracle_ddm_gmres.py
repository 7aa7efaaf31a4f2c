"""Pins of the one-step DDM preconditioner (Sec. 2, eq. ddm0, eq. pc and the
residual-in-PML property) and of restarted GMRES (Sec. 3)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import Problem, ddm, direct, gmres, operator, geometry, pool

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _prob(N, P, tile, n_ol, vel="random", omega=2 * np.pi * 4.0, seed=0):
    Ng = N + 2 * P
    if vel == "random":
        rng = np.random.default_rng(seed)
        vel = 1.0 + 0.3 * rng.random((Ng, Ng))
    elif vel == "const":
        vel = np.ones((Ng, Ng))
    return Problem(Nx=N, Ny=N, P=P, h=1.0 / N, omega=omega, k_ref=omega, velocity=vel,
                   tile=tile, n_ol=n_ol)


def test_local_residual_vanishes_on_physical_box_only():
    """Sec. 2: the local solution's residual is zero on the subdomain and
    nonzero in its PML.  Extending a local solution by zero, b - M E(u) vanishes
    on the box's physical nodes (tile + overlap + any global-layer part) and
    not in the box's own layer strips on interior sides."""
    prob = _prob(96, 8, 32, 4)
    P = ddm.OneStepDDM(prob)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    for i in (0, 4, 8):  # corner, centre, opposite corner
        box = P.boxes[i]
        u = P.local_solve(i, r)
        bx0, bx1 = box["bx"]; by0, by1 = box["by"]
        # local equation holds
        Ml = ddm.local_matrix(prob, box)
        b = ddm.restrict(r, box)
        assert np.linalg.norm(Ml @ u.ravel() - b.ravel()) <= 1e-12 * np.linalg.norm(b)
        Eu = np.zeros_like(r); Eu[by0:by1, bx0:bx1] = u
        Eb = np.zeros_like(r); Eb[by0:by1, bx0:bx1] = b
        res = Eb - operator.matvec(prob, Eu)
        phys = np.zeros(r.shape, bool)
        x0 = bx0 if box["ix"] == 0 else bx0 + 8
        x1 = bx1 if box["ix"] == prob.nbx - 1 else bx1 - 8
        y0 = by0 if box["iy"] == 0 else by0 + 8
        y1 = by1 if box["iy"] == prob.nby - 1 else by1 - 8
        phys[y0:y1, x0:x1] = True
        scale = np.abs(b).max()
        assert np.abs(res[phys]).max() <= 1e-10 * scale
        layer = np.zeros(r.shape, bool); layer[by0:by1, bx0:bx1] = True; layer &= ~phys
        assert np.abs(res[layer]).max() > 1e-3 * scale


def test_single_box_is_exact_inverse():
    """Nb = 1: the one box is the whole truncated domain, so P^-1 = M^-1 and
    GMRES converges in one iteration."""
    prob = _prob(32, 8, 32, 4)
    f = synth.gaussian_rhs(32, 8, [[0.3, 0.6]])
    P = ddm.OneStepDDM(prob)
    z = P.apply(f)
    u = direct.sparse_solve(prob, f)
    assert np.linalg.norm(z - u) <= 1e-12 * np.linalg.norm(u)
    x, info = gmres.solve(prob, f, tol=1e-10, precond=P)
    assert info["iters"] == 1


def test_preconditioner_linear_and_deterministic():
    prob = _prob(64, 8, 32, 4)
    P = ddm.OneStepDDM(prob)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    s = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    lhs = P.apply(a * r + b * s)
    rhs = a * P.apply(r) + b * P.apply(s)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)
    assert np.array_equal(P.apply(r), P.apply(r))
    # the sum covers every node: a residual supported on one tile only
    # produces exactly that box's local solution
    box = P.boxes[1]
    e = np.zeros_like(r); (tx0, tx1), (ty0, ty1) = box["tx"], box["ty"]
    e[ty0:ty1, tx0:tx1] = r[ty0:ty1, tx0:tx1]
    z = P.apply(e)
    u = P.local_solve(1, r)
    (bx0, bx1), (by0, by1) = box["bx"], box["by"]
    assert np.array_equal(z[by0:by1, bx0:bx1], u)
    z[by0:by1, bx0:bx1] = 0
    assert np.all(z == 0)


def test_gmres_plain_small_system():
    """Unpreconditioned GMRES with m >= n reaches the exact solve of a random
    complex system; CGS2 and MGS agree."""
    rng = np.random.default_rng(7)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for ortho in ("cgs2", "mgs"):
        x, info = gmres.gmres(lambda v: A @ v, lambda v: v, b, tol=1e-13, restart=n, ortho=ortho)
        assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
        assert info["iters"] <= n


def test_gmres_restarted_reaches_direct_solution():
    prob = _prob(16, 4, 8, 2)
    f = synth.gaussian_rhs(16, 4, [[0.4, 0.6]], width=2.5 / 16)
    u = direct.dense_solve(prob, f)
    P = ddm.OneStepDDM(prob)
    x, info = gmres.gmres(lambda v: operator.matvec(prob, v), P.apply, f, tol=1e-12, restart=5)
    assert info["relres_true"] <= 1e-12
    assert np.linalg.norm(x - u) <= 1e-9 * np.linalg.norm(u)
    x2, info2 = gmres.gmres(lambda v: operator.matvec(prob, v), P.apply, f, tol=1e-12, restart=5, ortho="mgs")
    assert abs(info2["iters"] - info["iters"]) <= 1


def test_gmres_started_again_from_a_cycle_end_takes_the_same_steps():
    """Restarted GMRES keeps no state across a cycle boundary but the
    iterate: a run started from the iterate handed to cycle_callback after
    cycle c ends bitwise where the uninterrupted run ends, after the
    remaining number of Arnoldi steps (what lets a long run be resumed)."""
    prob = _prob(32, 4, 8, 2)
    f = synth.gaussian_rhs(32, 4, [[0.4, 0.6]], width=2.5 / 32)
    A = lambda v: operator.matvec(prob, v)
    P = ddm.OneStepDDM(prob)
    ends = []
    x, info = gmres.gmres(A, P.apply, f, tol=1e-10, restart=3,
                          cycle_callback=lambda xc, it, cyc: ends.append((xc.copy(), it, cyc)))
    assert len(ends) == info["restarts"] >= 4
    assert np.array_equal(ends[-1][0], x)
    xc, it, cyc = ends[2]
    x2, info2 = gmres.gmres(A, P.apply, f, tol=1e-10, restart=3, x0=xc)
    assert np.array_equal(x2, x)
    assert it + info2["iters"] == info["iters"] and cyc + info2["restarts"] == info["restarts"]


def paper_sweep_band():
    """The equivalent sweeps n_iter / max(Nb_x, Nb_y) printed in the paper's
    Tables 1-5 (tests/golden/paper_sweeps.txt, each row checked against its
    own iteration count), and the band they span: from half the smallest to
    the largest (the paper's runs use thicker layers and tolerance 1e-10)."""
    rows = []
    with open(os.path.join(GOLDEN, "paper_sweeps.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, medium, nb, iters, sweeps = line.split()
                rows.append((t, medium, int(nb), int(iters), int(sweeps)))
    for t, _, nb, iters, sweeps in rows:
        assert abs(iters / nb - sweeps) <= 0.5 + 1e-9, (t, nb, iters, sweeps)
    printed = [r[4] for r in rows]
    return min(printed) / 2, max(printed)


def test_c1_oracle_iterations_and_golden():
    """128^2 constant medium, 2x2 boxes: GMRES(50) to 1e-8.  The paper's 2x2
    constant-medium run needs 9 iterations (5 equivalent sweeps) with a 30-cell
    layer at tolerance 1e-10 (Table 2); equivalent sweeps here must fall in the
    band of all its constant, layered and Marmousi runs (2..12)."""
    lo, hi = paper_sweep_band()
    assert (lo, hi) == (2, 12)
    w = synth.config("c1_128")
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    x, info = gmres.solve(prob, f, tol=w.tol, restart=w.restart)
    assert info["relres_true"] <= w.tol
    sweeps = info["iters"] / w.nb
    assert lo <= sweeps <= hi
    u = direct.banded_solve(prob, f)
    assert np.linalg.norm(x - u) <= 1e-6 * np.linalg.norm(u)
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        g = json.load(fh)
    assert info["iters"] == g["iters"]
    for (iy, ix, re, im) in g["samples"]:
        assert abs(u[iy, ix] - (re + 1j * im)) <= 1e-12 * np.abs(u).max()


def test_smoothing_function_properties():
    """beta_ij of the Remark after eq. pc (reading: product of quintic C^2
    ramps across each interior side's overlap + layer strip).  The paper fixes
    beta = 1 on the tile and 0 outside the box and asks for C^2: checked on a
    3x3 layout, where interior sides carry strips of n_ol + P = 12 nodes and
    global-boundary sides none (the edge tiles reach the boundary)."""
    prob = _prob(96, 8, 32, 4)
    bxs = geometry.boxes(prob)
    for i in (0, 4, 7):  # corner, centre, edge
        box = bxs[i]
        (bx0, bx1), (by0, by1) = box["bx"], box["by"]
        (tx0, tx1), (ty0, ty1) = box["tx"], box["ty"]
        beta = ddm.smoothing(box)
        assert beta.shape == (by1 - by0, bx1 - bx0)
        assert np.all(beta[ty0 - by0:ty1 - by0, tx0 - bx0:tx1 - bx0] == 1.0)
        strips = np.ones(beta.shape, bool)
        strips[ty0 - by0:ty1 - by0, tx0 - bx0:tx1 - bx0] = False
        assert np.all((beta[strips] > 0) & (beta[strips] < 1))
        # strips only on interior sides, each n_ol + P wide
        assert (tx0 - bx0) == (0 if box["ix"] == 0 else 12)
        assert (bx1 - tx1) == (0 if box["ix"] == prob.nbx - 1 else 12)
    # one axis: decreasing away from the tile, symmetric, values of the quintic
    w = ddm.ramp_weights(20, 40, 8, 52)
    assert np.all(np.diff(w[:12]) > 0) and np.all(np.diff(w[32:]) < 0)
    assert np.allclose(w[:12], w[32:][::-1], rtol=0, atol=1e-15)
    s = (np.arange(12) + 0.5) / 12  # distance from the tile edge, in strip widths
    assert np.allclose(w[32:], 1 - (10 * s**3 - 15 * s**4 + 6 * s**5), atol=1e-15)
    assert np.allclose(w[32:] + w[32:][::-1], 1.0, atol=1e-14)  # S(s) + S(1-s) = 1
    # C^2 at both strip ends: on a fine strip the first and second differences
    # (in units of the strip width) vanish at the tile edge and at the box edge
    L = 4000
    w = ddm.ramp_weights(0, 1, 0, 1 + L)[1:]
    d1 = np.diff(w) * L
    d2 = np.diff(w, 2) * L * L
    assert abs(d1[0]) < 1e-5 and abs(d1[-1]) < 1e-5
    # S''(s) ~ 60 s near the ends: at s = 1.5 / L, 90 / L, against an interior peak of ~5.77
    assert abs(d2[0]) < 100.0 / L and abs(d2[-1]) < 100.0 / L
    assert np.abs(d2).max() > 5.7
    assert np.abs(d1).max() > 1.8  # the quintic's largest slope is 15/8


def test_smoothed_preconditioner_weights_box_solutions():
    """With smoothing, a residual supported on one tile returns beta times that
    box's local solution: equal to it on the tile, reduced in the strips, zero
    outside the box; with a single box (Nb = 1) beta is 1 everywhere and the
    smoothed preconditioner is the unsmoothed one; GMRES with the smoothed
    preconditioner still reaches the direct solution."""
    prob = _prob(96, 8, 32, 4)
    Ps = ddm.OneStepDDM(prob, smooth=True)
    P0 = ddm.OneStepDDM(prob)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    box = Ps.boxes[4]
    (bx0, bx1), (by0, by1) = box["bx"], box["by"]
    (tx0, tx1), (ty0, ty1) = box["tx"], box["ty"]
    e = np.zeros_like(r)
    e[ty0:ty1, tx0:tx1] = r[ty0:ty1, tx0:tx1]
    u = P0.apply(e)[by0:by1, bx0:bx1]
    zs = Ps.apply(e)
    assert np.array_equal(zs[ty0:ty1, tx0:tx1], u[ty0 - by0:ty1 - by0, tx0 - bx0:tx1 - bx0])
    assert np.allclose(zs[by0:by1, bx0:bx1], ddm.smoothing(box) * u, rtol=0, atol=1e-15)
    out = zs.copy()
    out[by0:by1, bx0:bx1] = 0
    assert np.all(out == 0)
    one = _prob(32, 8, 32, 4)
    f1 = synth.gaussian_rhs(32, 8, [[0.3, 0.6]])
    assert np.array_equal(ddm.OneStepDDM(one, smooth=True).apply(f1), ddm.OneStepDDM(one).apply(f1))
    f = synth.gaussian_rhs(96, 8, [[0.4, 0.55]])
    x, info = gmres.solve(prob, f, tol=1e-10, precond=Ps)
    xd = direct.sparse_solve(prob, f)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_multistep_ddm_single_box_exact_and_neighbours():
    """eq. ddms: with one box there are no neighbours, so step 0 (the exact
    local solve of the whole truncated domain) is the solution and later
    steps add nothing; the neighbour sets of a 3x3 layout have 3, 5 and 8
    members at corners, edges and the centre."""
    prob = _prob(32, 8, 32, 4)
    f = synth.gaussian_rhs(32, 8, [[0.3, 0.6]])
    u, hist = ddm.multistep(prob, f, steps=3)
    assert np.linalg.norm(u - direct.sparse_solve(prob, f)) <= 1e-12 * np.linalg.norm(u)
    assert hist[0] <= 1e-12 and len(hist) == 3
    p3 = _prob(96, 8, 32, 4)
    assert [len(ddm.neighbours(p3, i)) for i in (0, 1, 4, 8)] == [3, 5, 8, 3]
    assert sorted(ddm.neighbours(p3, 4)) == [0, 1, 2, 3, 5, 6, 7, 8]


def test_multistep_ddm_is_richardson_with_the_one_step_preconditioner():
    """The step-(s+1) sources summed over the tiles equal the global residual
    of the running sum, because each local solution leaves no residual on its
    own tile (the local-residual property pinned above): so eq. ddms / eq. sum
    is the Richardson iteration u <- u + P^-1 (f - M u) with the one-step
    preconditioner.  The literal neighbour sums and the Richardson form agree
    to rounding over 6 steps on a 3x3 random medium; on a 2x2 constant medium
    the iteration reaches 1e-10 within 12 steps."""
    prob = _prob(96, 8, 32, 4, seed=3)
    f = synth.gaussian_rhs(96, 8, [[0.4, 0.55]])
    u, hist = ddm.multistep(prob, f, steps=6)
    P = ddm.OneStepDDM(prob)
    x = np.zeros_like(f)
    for s in range(6):
        x = x + P.apply(f - operator.matvec(prob, x))
    assert np.linalg.norm(u - x) <= 1e-11 * np.linalg.norm(x)
    assert all(b < a for a, b in zip(hist[1:], hist[2:])) and hist[-1] < 0.05 * hist[1]
    p2 = _prob(128, 16, 64, 8, vel="const", omega=2 * np.pi * 12.8)
    f2 = synth.gaussian_rhs(128, 16, [[0.3, 0.6]])
    u2, h2 = ddm.multistep(p2, f2, steps=12, tol=1e-10)
    assert h2[-1] <= 1e-10 and len(h2) <= 12
    assert np.linalg.norm(u2 - direct.sparse_solve(p2, f2)) <= 1e-8 * np.linalg.norm(u2)


def test_pooled_preconditioner_equals_serial_bitwise():
    """The process-pool form runs the same restriction, SuperLU solve and
    lexicographic sum as the serial form, so the two agree bitwise, with the
    default and with the low-fill SuperLU options, plain and smoothed; the two
    SuperLU orderings give the same exact local solves up to rounding."""
    prob = _prob(96, 8, 32, 4, seed=6)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(prob.k2().shape) + 1j * rng.standard_normal(prob.k2().shape)
    ref = {}
    for opts in (None, ddm.LOW_FILL):
        for smooth in (False, True):
            z0 = ddm.OneStepDDM(prob, smooth=smooth, splu_options=opts).apply(r)
            with pool.PooledOneStepDDM(prob, workers=3, smooth=smooth, splu_options=opts) as P:
                z1 = P.apply(r)
                z2 = P.apply(2 * r)
            assert np.array_equal(z0, z1)
            assert np.array_equal(z2, ddm.OneStepDDM(prob, smooth=smooth, splu_options=opts).apply(2 * r))
            ref[(opts is None, smooth)] = z0
    for smooth in (False, True):
        a, b = ref[(True, smooth)], ref[(False, smooth)]
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


def test_pooled_apply_many_equals_single_applies_bitwise():
    """Several residuals through one pooled application (each box's factor
    solving their local sources as the columns of one matrix) give, residual
    by residual, bitwise the serial preconditioner's result; fewer residuals
    than the pool's width work too, and more are refused."""
    prob = _prob(96, 8, 32, 4, seed=7)
    rng = np.random.default_rng(9)
    shape = prob.k2().shape
    rs = [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(3)]
    serial = ddm.OneStepDDM(prob, splu_options=ddm.LOW_FILL)
    want = [serial.apply(r) for r in rs]
    with pool.PooledOneStepDDM(prob, workers=3, splu_options=ddm.LOW_FILL, columns=3) as P:
        got = P.apply_many(rs)
        got2 = P.apply_many(rs[1:])
        one = P.apply(rs[2])
        with pytest.raises(ValueError):
            P.apply_many(rs + rs[:1])
    for a, b in zip(want, got):
        assert np.array_equal(a, b)
    assert np.array_equal(got2[0], want[1]) and np.array_equal(got2[1], want[2])
    assert np.array_equal(one, want[2])
