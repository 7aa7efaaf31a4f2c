"""GPU parity: the HIP library against the FP64 oracle on seeded inputs.

Tolerances.  FP64 paths (matvec, complex128 factors/sweeps) differ from the
oracle only by rounding order and by the local direct algorithm (block Schur
recursion vs sparse LU): relative 1e-10 for the preconditioner, 1e-13 for the
stencil.  complex64 factors/sweeps carry FP32 rounding (unit roundoff 6e-8)
amplified by the local condition numbers: compared box by box, the largest
entry error over each overlapping box relative to that box's largest value
(bars in tests/gpu_common.py, about 3x the measured errors).  Solutions: relative L2 <= 1e-6 against the direct
solution at relative residual <= 1e-8, FP64 iteration count equal to the
oracle's within +-1.
"""
import numpy as np
import pytest

import synth
from oracle import Problem, ddm, direct, gmres, operator
from tests.gpu_common import (C64_BOX_BAR, C64_BOX_BAR_WIDE, box_max_errors, gpu_ready, lib_problem, rand_c, rel,
                              small_problem)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_ready(), reason="needs a ROCm GPU")]

PLAIN, MIXED = 0, 1
# residual-history bars: largest relative difference per Arnoldi step between
# the library's and the oracle's residual estimates on the 96^2 problem of
# test_convergence_history_matches_oracle_step_by_step (measured 1.6e-8 with
# complex128 factors, 8.1e-5 with complex64 ones; bars about 4-6x those)
HIST_C128 = 1e-7
HIST_C64 = 3e-4


def _solver(prob, precision, restart=50, factor_format=0):
    from paper_1508_02897_amd.solver import Solver
    s = Solver(lib_problem(prob, precision, factor_format), prob.velocity, device=0,
               restart=restart)
    s.factor()
    return s


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_matvec_matches_oracle():
    prob = small_problem(N=96, P=8)
    from paper_1508_02897_amd.solver import Solver
    s = Solver(lib_problem(prob, PLAIN), prob.velocity)
    x = rand_c(prob.k2().shape, 11)
    y = _np(s.matvec(x))
    ref = operator.matvec(prob, x)
    print("matvec rel err", rel(y, ref))
    assert rel(y, ref) <= 1e-13


@pytest.mark.parametrize("shape", [(96, 8, 32, 4), (128, 16, 64, 8), (80, 8, 40, 4),
                                   (384, 16, 128, 8)])
def test_apply_plain_matches_oracle(shape):
    N, P, tile, n_ol = shape
    prob = small_problem(N=N, P=P, tile=tile, n_ol=n_ol, seed=N)
    s = _solver(prob, PLAIN)
    r = rand_c(prob.k2().shape, 3)
    z = _np(s.apply_precond(r))
    ref = ddm.OneStepDDM(prob).apply(r)
    e = rel(z, ref)
    print(f"apply c128 {shape} rel err {e:.3e}")
    assert e <= 1e-10


@pytest.mark.parametrize("shape", [(96, 8, 32, 4), (128, 16, 64, 8), (384, 16, 128, 8)])
def test_apply_mixed_matches_oracle(shape):
    N, P, tile, n_ol = shape
    prob = small_problem(N=N, P=P, tile=tile, n_ol=n_ol, seed=N)
    s = _solver(prob, MIXED)
    r = rand_c(prob.k2().shape, 3)
    z = _np(s.apply_precond(r))
    ref = ddm.OneStepDDM(prob).apply(r)
    e = rel(z, ref)
    eb = box_max_errors(z, ref, prob)
    print(f"apply c64 {shape} rel err {e:.3e} box max err {eb.max():.3e} (median {np.median(eb):.3e})")
    assert eb.max() <= C64_BOX_BAR


def test_apply_deterministic_and_linear():
    prob = small_problem(N=96, P=8)
    s = _solver(prob, PLAIN)
    r = rand_c(prob.k2().shape, 5)
    q = rand_c(prob.k2().shape, 6)
    z1 = _np(s.apply_precond(r))
    z2 = _np(s.apply_precond(r))
    assert np.array_equal(z1, z2)
    a = 0.7 - 0.2j
    zl = _np(s.apply_precond(a * r + q))
    zq = _np(s.apply_precond(q))
    assert rel(zl, a * z1 + zq) <= 1e-12


def test_single_box_exact_one_iteration():
    prob = small_problem(N=32, P=8, tile=32, n_ol=4, seed=9)
    s = _solver(prob, PLAIN)
    f = synth.gaussian_rhs(32, 8, [[0.4, 0.6]])
    z = _np(s.apply_precond(f))
    u = direct.sparse_solve(prob, f)
    assert rel(z, u) <= 1e-11
    x, info = s.solve(f, tol=1e-10)
    assert info["iters"] == 1
    assert rel(_np(x), u) <= 1e-10


def test_c1_solve_plain_matches_oracle():
    w = synth.config("c1_128")
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    s = _solver(prob, PLAIN)
    x, info = s.solve(f, tol=w.tol, restart=w.restart)
    x = _np(x)
    _, oinfo = gmres.solve(prob, f, tol=w.tol, restart=w.restart)
    u = direct.banded_solve(prob, f)
    print("gpu", info, "oracle iters", oinfo["iters"], "relL2", rel(x, u))
    assert info["relres_true"] <= w.tol
    assert abs(info["iters"] - oinfo["iters"]) <= 1
    assert rel(x, u) <= 1e-6
    r = f - operator.matvec(prob, x)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= w.tol


def test_c1_solve_mixed_matches_oracle():
    w = synth.config("c1_128")
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    s = _solver(prob, MIXED)
    x, info = s.solve(f, tol=w.tol, restart=w.restart)
    x = _np(x)
    u = direct.banded_solve(prob, f)
    _, oinfo = gmres.solve(prob, f, tol=w.tol, restart=w.restart)
    print("gpu mixed", info, "oracle iters", oinfo["iters"], "relL2", rel(x, u))
    assert info["relres_true"] <= w.tol
    assert rel(x, u) <= 1e-6
    r = f - operator.matvec(prob, x)
    assert np.linalg.norm(r) / np.linalg.norm(f) <= w.tol
    assert abs(info["iters"] - oinfo["iters"]) <= 1


def test_small_random_solve_both_precisions():
    prob = small_problem(N=96, P=8, tile=32, n_ol=4, seed=21)
    f = synth.gaussian_rhs(96, 8, [[0.3, 0.4], [0.7, 0.66]])
    u = direct.sparse_solve(prob, f)
    _, oinfo = gmres.solve(prob, f, tol=1e-8, restart=20)
    for prec in (PLAIN, MIXED):
        s = _solver(prob, prec, restart=20)
        x, info = s.solve(f, tol=1e-8, restart=20)
        print(prec, info, oinfo["iters"])
        assert info["relres_true"] <= 1e-8
        assert rel(_np(x), u) <= 1e-6
        assert abs(info["iters"] - oinfo["iters"]) <= 1


def test_apply_mixed_sweep_variants_agree():
    """Dense complex64 format: the wave-structured sweep and the
    one-row-per-thread sweep (several workgroup sizes) compute the same
    preconditioner as the symmetric-packed format (boxes 168/176 wide, as at
    4096^2)."""
    from paper_1508_02897_amd import hddm as H
    prob = small_problem(N=384, P=16, tile=128, n_ol=8, seed=3)
    r = rand_c(prob.k2().shape, 8)
    sp = _solver(prob, MIXED)
    z_pk = _np(sp.apply_precond(r))
    H.hddm_tune(sp.ctx, 1, 0, 0)  # packed, register cap for two workgroups per CU
    z_pk2 = _np(sp.apply_precond(r))
    print("packed one vs two per CU", rel(z_pk2, z_pk))
    assert np.array_equal(z_pk, z_pk2)
    s = _solver(prob, MIXED, factor_format=1)
    H.hddm_tune(s.ctx, H.SWEEP_WAVE, 0, 0)
    z_wave = _np(s.apply_precond(r))
    e = rel(z_pk, z_wave)
    print("packed vs dense wave sweep", e)
    assert e <= 1e-5
    for th in (0, 448, 1024):
        H.hddm_tune(s.ctx, H.SWEEP_ROW, th, 0)
        z_row = _np(s.apply_precond(r))
        e = rel(z_wave, z_row)
        print("wave vs row sweep", th, e)
        assert e <= 1e-5


@pytest.mark.parametrize("factor_format", [0, 1])
def test_mfma_and_vector_factors_agree(factor_format):
    """The MFMA complex64 factor and the vector-FMA complex64 factor give the
    same preconditioner to FP32 rounding, in the packed and the dense format
    (boxes 104 wide with a ragged last 16-block, and 168/176 wide)."""
    from paper_1508_02897_amd import hddm as H
    for shape in ((128, 16, 64, 8), (384, 16, 128, 8)):
        N, P, tile, n_ol = shape
        prob = small_problem(N=N, P=P, tile=tile, n_ol=n_ol, seed=N + 1)
        r = rand_c(prob.k2().shape, 9)
        s = _solver(prob, MIXED, factor_format=factor_format)
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_AUTO)
        s.factor()
        z_mfma = _np(s.apply_precond(r))
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_VECTOR)
        s.factor()
        z_vec = _np(s.apply_precond(r))
        ref = ddm.OneStepDDM(prob).apply(r)
        print(shape, factor_format, "mfma vs vector", rel(z_mfma, z_vec), "mfma vs oracle",
              rel(z_mfma, ref), "box max", box_max_errors(z_mfma, ref, prob).max(),
              box_max_errors(z_mfma, z_vec, prob).max())
        assert rel(z_mfma, z_vec) <= 1e-4
        assert box_max_errors(z_mfma, ref, prob).max() <= C64_BOX_BAR


@pytest.mark.parametrize("factor_format", [0, 1])
def test_register_and_memory_mfma_factors_bitwise_equal(factor_format):
    """The register-resident MFMA factor repeats the memory-working-matrix MFMA
    factor's arithmetic in the same order: the stored factors are bitwise
    equal (packed and dense format; boxes 104 wide with a ragged last
    16-block, 168/176 wide, and a single 192-wide box)."""
    import torch
    from paper_1508_02897_amd import hddm as H
    for shape in ((128, 16, 64, 8), (384, 16, 128, 8), (160, 16, 160, 0)):
        N, P, tile, n_ol = shape
        prob = small_problem(N=N, P=P, tile=tile, n_ol=n_ol, seed=N + 7)
        s = _solver(prob, MIXED, factor_format=factor_format)
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_MFMA_REGS)
        s.factor()
        torch.cuda.synchronize()
        g_reg = s.factor_buf.clone()
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_MFMA_MEM)
        s.factor()
        torch.cuda.synchronize()
        same = torch.equal(g_reg, s.factor_buf)
        print(shape, factor_format, "register vs memory MFMA factor bitwise equal:", same)
        assert same


@pytest.mark.parametrize("factor_format", [0, 1])
def test_symmetric_elimination_factor(factor_format):
    """The MFMA factor that eliminates on the upper tiles only (the symmetric
    form of Gauss-Jordan) stores the same inverses as the full elimination to
    FP32 rounding, with the same pivots; the dense format it writes is
    symmetric to rounding, and its preconditioner meets the oracle at the complex64 box
    bar (boxes 104 wide with a ragged last 16-block, 168/176 wide, and a
    single 192-wide box)."""
    import torch
    from paper_1508_02897_amd import hddm as H
    for shape in ((128, 16, 64, 8), (384, 16, 128, 8), (160, 16, 160, 0)):
        N, P, tile, n_ol = shape
        prob = small_problem(N=N, P=P, tile=tile, n_ol=n_ol, seed=N + 11)
        r = rand_c(prob.k2().shape, 5)
        s = _solver(prob, MIXED, factor_format=factor_format)
        nb = prob.nbx * prob.nby
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_MFMA_REGS)
        s.factor()
        torch.cuda.synchronize()
        g_full = s.factor_buf.clone().view(torch.complex64)
        piv_full = H.hddm_factor_pivots(s.ctx, nb)
        z_full = _np(s.apply_precond(r))
        H.hddm_tune(s.ctx, 0, 0, H.FACTOR_MFMA_SYM)
        s.factor()
        torch.cuda.synchronize()
        g_sym = s.factor_buf.view(torch.complex64)
        piv_sym = H.hddm_factor_pivots(s.ctx, nb)
        z_sym = _np(s.apply_precond(r))
        ref = ddm.OneStepDDM(prob).apply(r)
        gerr = float((g_sym - g_full).abs().max() / g_full.abs().max())
        bm = box_max_errors(z_sym, ref, prob).max()
        print(shape, factor_format, "factor max rel diff", gerr, "pivots", piv_sym.min(),
              piv_sym.max(), "apply vs full elimination", rel(z_sym, z_full), "box max vs oracle", bm)
        assert gerr <= 1e-4
        assert np.allclose(piv_sym, piv_full, rtol=1e-4, atol=0)
        assert rel(z_sym, z_full) <= 1e-4
        assert bm <= (C64_BOX_BAR if shape[2] < 160 else C64_BOX_BAR_WIDE)
        if factor_format == 1:  # dense: G_0 of the first box written in full, symmetric
            _, _, boxes = H.hddm_geometry(s.ctx)
            mx = int(boxes[0][1] - boxes[0][0])
            G0 = g_sym[:mx * mx].cpu().numpy().reshape(mx, mx)
            assert np.abs(G0 - G0.T).max() <= 1e-5 * np.abs(G0).max()


@pytest.mark.parametrize("precision", [PLAIN, MIXED])
def test_gram_cgs2_matches_explicit_cgs2(precision):
    """CGS2 with the second projection taken from the Gram matrix (two passes
    over the basis) reproduces explicit CGS2 (four passes): same iteration
    count within 1, same solution to the solve tolerance, on the 128^2
    workload and on a 96^2 random medium with restarts."""
    cases = []
    w = synth.config("c1_128")
    cases.append((Problem.from_workload(w), synth.rhs_for(w), 50))
    p2 = small_problem(N=96, P=8, tile=32, n_ol=4, seed=21)
    cases.append((p2, synth.gaussian_rhs(96, 8, [[0.3, 0.4], [0.7, 0.66]]), 8))
    for prob, f, m in cases:
        s = _solver(prob, precision, restart=m)
        x0, i0 = s.solve(f, tol=1e-10, restart=m, ortho=0)
        x1, i1 = s.solve(f, tol=1e-10, restart=m, ortho=1)
        x0, x1 = _np(x0), _np(x1)
        print(precision, m, i0, i1, rel(x1, x0))
        assert abs(i0["iters"] - i1["iters"]) <= 1
        assert i1["relres_true"] <= 1e-10
        assert rel(x1, x0) <= 1e-7


@pytest.mark.parametrize("n_ol,P", [(0, 16), (50, 30)])
def test_overlap_and_pml_widths_match_oracle(n_ol, P):
    """The overlap/PML-width study's extremes on a 320^2 three-layer problem
    with 2x2 tiles of 160: no overlap with a 16-cell layer (boxes 176-192
    wide, packed factors) and an overlap of 50 with a 30-cell layer (boxes
    270 wide, dense factors and the generic kernels).  The preconditioner
    against the oracle's: complex128 (1e-10) where the boxes fit its factor
    (at most 208 wide), else complex64 (per box); complex64 FGMRES(50) to 1e-8
    against the oracle's GMRES iteration count (+-1) and the direct solution
    (relative L2 <= 1e-6)."""
    w = synth.Workload(name="widths", N=320, P=P, tile=160, n_ol=n_ol, ppw=10.0, c_min=1.0,
                       medium="layered", medium_seed=3, n_sources=1, source_seed=3)
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    r = rand_c(prob.k2().shape, 31)
    zo = ddm.OneStepDDM(prob).apply(r)
    side = 160 + n_ol + 2 * P  # corner boxes of the 2x2 layout
    prec, bar = (PLAIN, 1e-10) if side <= 208 else (MIXED, C64_BOX_BAR_WIDE)
    s = _solver(prob, prec)
    za = _np(s.apply_precond(r))
    e_apply = rel(za, zo) if prec == PLAIN else box_max_errors(za, zo, prob).max()
    s.close()
    s = _solver(prob, MIXED)
    x, info = s.solve(f, tol=1e-8, restart=50)
    x = _np(x)
    s.close()
    _, oinfo = gmres.solve(prob, f, tol=1e-8, restart=50)
    u = direct.sparse_solve(prob, f)
    e = rel(x, u)
    print(f"n_ol {n_ol} P {P}: apply vs oracle {e_apply:.2e}; {info} oracle iters "
          f"{oinfo['iters']}; rel L2 {e:.2e}")
    assert e_apply <= bar
    assert info["relres_true"] <= 1e-8
    assert abs(info["iters"] - oinfo["iters"]) <= 1
    assert e <= 1e-6


def test_smoothing_function_matches_oracle():
    """The smoothing function of the Remark after eq. pc (beta_ij on every
    local solution before the sum) against the oracle's, on a 96^2 random
    medium with 3x3 boxes (interior, edge and corner strips): complex128
    preconditioner 1e-10, complex64 single and block form per box,
    and complex64 FGMRES to 1e-8 against the oracle's GMRES with the smoothed
    preconditioner (iterations +-1, direct solution 1e-6).  With smoothing off
    again the result is the plain sum's, bitwise."""
    from paper_1508_02897_amd import hddm as H
    prob = small_problem(N=96, P=8, tile=32, n_ol=4, seed=13)
    r = rand_c(prob.k2().shape, 41)
    zo = ddm.OneStepDDM(prob, smooth=True).apply(r)
    zo_plain = ddm.OneStepDDM(prob).apply(r)
    s = _solver(prob, PLAIN)
    z_plain = _np(s.apply_precond(r))
    H.hddm_set_smoothing(s.ctx, True)
    e128 = rel(_np(s.apply_precond(r)), zo)
    H.hddm_set_smoothing(s.ctx, False)
    assert np.array_equal(_np(s.apply_precond(r)), z_plain)
    s.close()
    s = _solver(prob, MIXED)
    H.hddm_set_smoothing(s.ctx, True)
    e64 = box_max_errors(_np(s.apply_precond(r)), zo, prob).max()
    eblk = box_max_errors(_np(s.apply_precond_block(np.stack([r, 2 * r])))[1], 2 * zo, prob).max()
    f = synth.gaussian_rhs(96, 8, [[0.35, 0.6]])
    x, info = s.solve(f, tol=1e-8, restart=30)
    x = _np(x)
    s.close()
    _, oinfo = gmres.solve(prob, f, tol=1e-8, restart=30, precond=ddm.OneStepDDM(prob, smooth=True))
    e = rel(x, direct.sparse_solve(prob, f))
    print(f"smoothing: c128 {e128:.2e} c64 {e64:.2e} block {eblk:.2e}; smoothed vs plain "
          f"{rel(zo, zo_plain):.2e}; {info} oracle iters {oinfo['iters']}; rel L2 {e:.2e}")
    assert rel(zo, zo_plain) > 1e-6  # the weights do change the preconditioner
    assert e128 <= 1e-10
    assert e64 <= C64_BOX_BAR and eblk <= C64_BOX_BAR
    assert info["relres_true"] <= 1e-8
    assert abs(info["iters"] - oinfo["iters"]) <= 1
    assert e <= 1e-6


def test_multistep_ddm_solver_matches_oracle():
    """The iterative multi-step DDM (eq. ddms) run as a solver against the
    oracle's literal neighbour-residual steps: after 6 steps on a 96^2 random
    medium with 3x3 boxes the complex128 sums agree to 1e-10 (and the
    residuals after each step count); on a 128^2 constant medium with 2x2
    boxes the complex64 solver reaches 1e-8 in the oracle's number of steps
    (+-1) and matches the direct solution to 1e-6."""
    prob = small_problem(N=96, P=8, tile=32, n_ol=4, seed=17)
    f = synth.gaussian_rhs(96, 8, [[0.4, 0.55]])
    uo, ho = ddm.multistep(prob, f, steps=6)
    s = _solver(prob, PLAIN)
    x, info = s.ddm_solve(f, max_steps=6, tol=0.0, raise_on_noconv=False)
    x = _np(x)
    s.close()
    e6 = rel(x, uo)
    print(f"6 steps: vs oracle {e6:.2e}; relres {info['relres_est']:.4e} oracle {ho[-1]:.4e}")
    assert info["iters"] == 6 and e6 <= 1e-10
    assert abs(info["relres_est"] - ho[-1]) <= 1e-8 * ho[-1]
    assert abs(info["relres_true"] - ho[-1]) <= 1e-8 * ho[-1]
    w = synth.config("c1_128")
    p2 = Problem.from_workload(w)
    f2 = synth.rhs_for(w)
    _, h2 = ddm.multistep(p2, f2, steps=200, tol=1e-8)
    s = _solver(p2, MIXED)
    x2, i2 = s.ddm_solve(f2, max_steps=200, tol=1e-8)
    x2 = _np(x2)
    s.close()
    e2 = rel(x2, direct.sparse_solve(p2, f2))
    print(f"c1: {i2} oracle steps {len(h2)} rel L2 {e2:.2e}")
    assert i2["relres_true"] <= 1e-8 and abs(i2["iters"] - len(h2)) <= 1 and e2 <= 1e-6


@pytest.mark.parametrize("restart", [20, 5])
def test_convergence_history_matches_oracle_step_by_step(restart):
    """The residual estimate |gamma_{j+1}| / |b| after every Arnoldi step
    (hddm_solve_history, Sec. 3's restarted GMRES) against the oracle's
    history on the same problem, step by step: complex128 factors, then
    complex64 factors in the single and the block form (three sources, each
    against its own oracle run).  With restart 5 the histories cross several
    cycle ends, where both sides start again from the true residual."""
    prob = small_problem(N=96, P=8, tile=32, n_ol=4, seed=21)
    srcs = [[[0.3, 0.4]], [[0.7, 0.66]], [[0.52, 0.2]]]
    F = [synth.gaussian_rhs(96, 8, c) for c in srcs]
    oh = []
    for f in F:
        _, oinfo = gmres.solve(prob, f, tol=1e-8, restart=restart)
        oh.append(np.array(oinfo["history"]))
        assert len(oh[-1]) == oinfo["iters"]

    def worst(h, o):
        n = min(len(h), len(o))
        return float((np.abs(h[:n] - o[:n]) / o[:n]).max())

    for prec, bar in ((PLAIN, HIST_C128), (MIXED, HIST_C64)):
        s = _solver(prob, prec, restart=restart)
        _, info = s.solve(F[0], tol=1e-8, restart=restart)
        h = s.history()
        d = worst(h, oh[0])
        print("single", prec, restart, len(h), len(oh[0]), d)
        assert len(h) == info["iters"] and abs(len(h) - len(oh[0])) <= 1
        assert d <= bar
        if prec == MIXED:
            _, infos = s.solve_block(np.stack(F), tol=1e-8, restart=restart)
            for k in range(len(F)):
                hk = s.history(k)
                dk = worst(hk, oh[k])
                print("block", k, restart, len(hk), len(oh[k]), dk)
                assert len(hk) == infos[k]["iters"] and abs(len(hk) - len(oh[k])) <= 1
                assert dk <= bar
        s.close()
