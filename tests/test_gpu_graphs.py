"""Graph replay of the single-form preconditioner application: every form
(complex64 packed and dense factors, complex128) as one graph launch against
the same kernels launched one by one.  Each replay gets other arguments, with
eager launches and synchronisations between replays and two replays back to
back; every result must be bitwise the eager one, and a solve must take the
same iterations to bitwise the same solution."""
import numpy as np
import pytest

import synth
from tests.gpu_common import gpu_ready, lib_problem, rand_c, small_problem

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a ROCm GPU")]


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("precision,fmt", [(1, 0), (1, 1), (0, 1)])
def test_single_apply_graph_replays_match_eager(precision, fmt):
    import torch
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import Solver
    prob = small_problem(N=128, P=16, tile=64, n_ol=8, seed=21)
    s = Solver(lib_problem(prob, precision, fmt), prob.velocity, device=0, restart=10)
    s.factor()
    Rs = [rand_c(prob.k2().shape, 500 + t) for t in range(4)]
    H.hddm_use_graphs(s.ctx, False)
    eager = [_np(s.apply_precond(R)) for R in Rs]
    H.hddm_use_graphs(s.ctx, True)
    for t, R in enumerate(Rs):
        assert np.array_equal(_np(s.apply_precond(R)), eager[t]), t
        H.hddm_use_graphs(s.ctx, False)
        assert np.array_equal(_np(s.apply_precond(Rs[(t + 1) % 4])), eager[(t + 1) % 4])
        H.hddm_use_graphs(s.ctx, True)
    ra = torch.from_numpy(Rs[1]).to("cuda:0")
    rb = torch.from_numpy(Rs[2]).to("cuda:0")
    za = s.apply_precond(ra)
    zb = s.apply_precond(rb)
    assert np.array_equal(_np(za), eager[1]) and np.array_equal(_np(zb), eager[2])
    b = synth.gaussian_rhs(128, 16, [[0.4, 0.6]])
    xg, ig = s.solve(b, tol=1e-8, restart=10)
    xg = _np(xg)
    H.hddm_use_graphs(s.ctx, False)
    xe, ie = s.solve(b, tol=1e-8, restart=10)
    xe = _np(xe)
    assert ig["iters"] == ie["iters"] and np.array_equal(xg, xe)
    s.close()
