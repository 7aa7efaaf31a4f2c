"""The line factor inverts every Schur complement S_j of a box by Gauss-Jordan
without pivoting (local direct solves, Sec. 3).  Checked here in FP64 on
176-wide interior and 168-wide corner boxes of the serving and benchmark
media, against LAPACK's pivoted inverse: the unpivoted inverses agree, the
recorded pivots are the ratios of leading principal minors (a property of
unpivoted elimination, checked with LAPACK determinants), and no pivot falls
far below the diagonal entry it started from (|p_k| / |S_j(k,k)| >= 0.3: no
cancellation, so no growth that pivoting would have to avoid).  kh is the largest
wave number times h over the box (c = 0.8 at 8 ppw in the random medium
gives kh = 0.785, the top of the range the serving mix uses)."""
import numpy as np
import pytest

import synth
from oracle import Problem, ddm
from oracle.geometry import boxes
from tests.unpivoted import schur_recursion

# (generator, ppw, medium seed, correlation length, box): random medium at
# 8 ppw (c_min = 0.8, the serving mix's coarsest) on an interior box;
# three-layer at 12 ppw (c_min = 1.0) on a corner box
MEDIA = [("random", 8.0, 0, 20.0, 5), ("layered", 12.0, 4, 20.0, 0)]


def _workload(kind, ppw, seed, corr):
    return synth.Workload(name=f"pivots_{kind}_{ppw:g}", N=512, P=16, tile=128, n_ol=8, ppw=ppw,
                          c_min=0.8 if kind == "random" else 1.0, medium=kind, medium_seed=seed,
                          corr_len_h=corr)


@pytest.mark.parametrize("kind,ppw,seed,corr,ibox", MEDIA)
def test_unpivoted_inversions_match_lapack(kind, ppw, seed, corr, ibox):
    w = _workload(kind, ppw, seed, corr)
    prob = Problem.from_workload(w)
    kh = float(np.sqrt(prob.k2().max()) * prob.h)
    for i in (ibox,):  # 5: interior box (176 x 176), 0: corner box (168 x 168)
        box = boxes(prob)[i]
        mx = box["bx"][1] - box["bx"][0]
        my = box["by"][1] - box["by"][0]
        M = ddm.local_matrix(prob, box)
        worst_inv = 0.0
        pmin, pmax = np.inf, 0.0
        for j, S, G, piv in schur_recursion(M, mx, my):
            Gl = np.linalg.inv(S)  # LAPACK, partial pivoting
            worst_inv = max(worst_inv, np.abs(G - Gl).max() / np.abs(Gl).max())
            rp = np.abs(piv) / np.abs(np.diag(S))  # pivot relative to its diagonal entry
            pmin = min(pmin, rp.min())
            pmax = max(pmax, rp.max())
            if j in (0, my // 2, my - 1):
                # unpivoted elimination: pivot k = det(S[:k+1, :k+1]) / det(S[:k, :k])
                for k in (1, mx // 3, mx - 1):
                    s1, l1 = np.linalg.slogdet(S[:k + 1, :k + 1])
                    s0, l0 = np.linalg.slogdet(S[:k, :k])
                    ratio = (s1 / s0) * np.exp(l1 - l0)
                    assert abs(piv[k] - ratio) <= 1e-9 * abs(ratio)
        print(f"{kind} {ppw:g} ppw kh {kh:.3f} box {i} ({mx}x{my}): unpivoted vs LAPACK "
              f"inverse {worst_inv:.1e}, relative pivots |p_k| / |S_j(k,k)| in "
              f"[{pmin:.3f}, {pmax:.3f}]")
        assert worst_inv <= 1e-11
        assert pmin >= 0.3  # no cancellation on the diagonal (measured 0.53 - 0.57)
