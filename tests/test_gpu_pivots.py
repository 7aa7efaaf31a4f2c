"""The line factor's pivot diagnostic (hddm_factor_pivots) against an FP64
NumPy reference of the same unpivoted elimination (tests/unpivoted.py, on the
oracle's local matrices): per box, the smallest and largest relative pivot
|p_k| / |S_j(k,k)| over all x-lines, for the complex128 factor, the complex64
MFMA factors (working matrix in registers, in memory) and the complex64
vector factor, on a 384^2 layout of 3x3 boxes 168/176 wide."""
import numpy as np
import pytest

from oracle import ddm
from oracle.geometry import boxes
from tests.gpu_common import gpu_ready, lib_problem, small_problem
from tests.unpivoted import schur_recursion

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a ROCm GPU")]

PLAIN, MIXED = 0, 1
CHECK_BOXES = (0, 1, 4)  # corner, edge, interior


def _reference(prob):
    out = {}
    bxs = boxes(prob)
    for i in CHECK_BOXES:
        b = bxs[i]
        mx, my = b["bx"][1] - b["bx"][0], b["by"][1] - b["by"][0]
        lo, hi = np.inf, 0.0
        for _, S, _, piv in schur_recursion(ddm.local_matrix(prob, b), mx, my):
            r = np.abs(piv) / np.abs(np.diag(S))
            lo, hi = min(lo, r.min()), max(hi, r.max())
        out[i] = (lo, hi)
    return out


def test_factor_pivots_match_fp64_reference():
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import Solver
    prob = small_problem(N=384, P=16, tile=128, n_ol=8, seed=17)
    ref = _reference(prob)
    cases = [(PLAIN, H.FACTOR_AUTO, 1e-5), (MIXED, H.FACTOR_AUTO, 2e-3),
             (MIXED, H.FACTOR_MFMA_MEM, 2e-3), (MIXED, H.FACTOR_MFMA_REGS, 2e-3),
             (MIXED, H.FACTOR_VECTOR, 2e-3)]
    for prec, fvar, tol in cases:
        s = Solver(lib_problem(prob, prec), prob.velocity, device=0, restart=3)
        with pytest.raises(H.HddmError) as e:  # before the factorisation
            H.hddm_factor_pivots(s.ctx, 9)
        assert e.value.status == H.HDDM_ESTATE
        H.hddm_tune(s.ctx, 0, 0, fvar)
        s.factor()
        pv = H.hddm_factor_pivots(s.ctx, 9)
        for i in CHECK_BOXES:
            lo, hi = ref[i]
            print(f"precision {prec} factor variant {fvar} box {i}: kernel [{pv[i, 0]:.6f}, "
                  f"{pv[i, 1]:.6f}] reference [{lo:.6f}, {hi:.6f}]", flush=True)
            assert abs(pv[i, 0] - lo) <= tol * lo
            assert abs(pv[i, 1] - hi) <= tol * hi
        assert np.all(pv[:, 0] > 0.3) and np.all(np.isfinite(pv))
        if prec == MIXED and fvar == H.FACTOR_AUTO:
            # a context sharing the factor reports nothing of its own
            t = Solver(lib_problem(prob, prec), prob.velocity, device=0, restart=3, share_from=s)
            with pytest.raises(H.HddmError) as e:
                H.hddm_factor_pivots(t.ctx, 9)
            assert e.value.status == H.HDDM_ESTATE
            t.close()
        s.close()


def test_nested_dissection_reports_no_pivots():
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import Solver
    prob = small_problem(N=96, P=8, tile=32, n_ol=4, seed=3)
    s = Solver(lib_problem(prob, MIXED, H.FORMAT_NESTED_DISSECTION), prob.velocity, device=0,
               restart=3)
    s.factor()
    with pytest.raises(H.HddmError) as e:
        H.hddm_factor_pivots(s.ctx, 9)
    assert e.value.status == H.HDDM_EINVAL
    s.close()
