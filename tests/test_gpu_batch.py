"""Several problems in one launch sequence (the serving path): the
preconditioner of eq. pc applied for contexts of different grids, media and
wave numbers with one fused block sweep over all their boxes, and the solver
session that advances their block FGMRES (Sec. 3) one round at a time with
problems joining while others iterate.  Each problem's result is bitwise its
own stand-alone block apply / block solve (same kernels per box and per
right-hand side, same order), and the batch is checked against the oracle's
preconditioner box by box."""
import numpy as np
import pytest

import synth
from oracle import Problem, ddm
from tests.gpu_common import C64_BOX_BAR, box_max_errors, gpu_ready, rand_c

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a ROCm GPU")]

MIXED = 1


def _workload(N, seed, ppw):
    kind = "random" if seed < 4 else "layered"
    return synth.Workload(name=f"batch_{N}_{seed}", N=N, P=16, tile=128, n_ol=8, ppw=ppw,
                          c_min=0.8 if kind == "random" else 1.0, medium=kind, medium_seed=seed,
                          corr_len_h=20.0)


def _solver(w, restart=3):
    from paper_1508_02897_amd.solver import Solver, problem_from_workload
    s = Solver(problem_from_workload(w, MIXED), synth.medium_for(w), device=0, restart=restart)
    s.factor()
    return s


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def test_batch_apply_equals_each_block_apply_and_oracle():
    import torch
    from paper_1508_02897_amd import hddm as H
    ws = [_workload(384, 1, 10.0), _workload(256, 5, 12.0), _workload(512, 2, 8.0)]
    nr = [3, 1, 5]
    ss = [_solver(w) for w in ws]
    R = [torch.from_numpy(np.stack([rand_c((w.Ng, w.Ng), 900 + 10 * i + k) for k in range(n)]))
         .to("cuda") for i, (w, n) in enumerate(zip(ws, nr))]
    ref = [s.apply_precond_block(r).cpu().numpy() for s, r in zip(ss, R)]
    Z = [torch.empty_like(r) for r in R]
    bufs = [s.ensure_block(n, 1)[0] for s, n in zip(ss, nr)]
    for rep in range(2):  # graph built, then replayed
        for z in Z:
            z.zero_()
        H.hddm_apply_precond_batch([s.ctx for s in ss], [r.data_ptr() for r in R],
                                   [w.Ng * w.Ng for w in ws], [z.data_ptr() for z in Z],
                                   [w.Ng * w.Ng for w in ws], nr, [b.data_ptr() for b in bufs],
                                   [b.numel() for b in bufs], _stream())
        torch.cuda.synchronize()
        for i in range(3):
            assert np.array_equal(Z[i].cpu().numpy(), ref[i]), (rep, i)
    # one column of each problem against the oracle's preconditioner
    for i, w in enumerate(ws):
        prob = Problem.from_workload(w)
        zo = ddm.OneStepDDM(prob).apply(R[i][0].cpu().numpy())
        e = box_max_errors(ref[i][0], zo, prob).max()
        print(f"batch problem {i} ({w.N}^2): box max err vs oracle {e:.2e}", flush=True)
        assert e <= C64_BOX_BAR
    for s in ss:
        s.close()


def test_batch_rejects_mixed_shapes():
    import torch
    from paper_1508_02897_amd import hddm as H
    from paper_1508_02897_amd.solver import Solver, make_problem
    a = _solver(_workload(256, 1, 10.0))
    N = 96
    vel = synth.random_medium(N, 8, corr_len_h=6.0, seed=1)
    om = 2 * np.pi * 0.8 * N / 10.0
    b = Solver(make_problem(N, N, 8, 32, 4, 1.0 / N, om, om, precision=MIXED), vel, device=0)
    b.factor()  # boxes of 52/56: another tile-block width
    with pytest.raises(H.HddmError) as e:
        H.hddm_apply_precond_batch([a.ctx, b.ctx], [256, 256], [1, 1], [256, 256], [1, 1], [1, 1],
                                   [256, 256], [1 << 40, 1 << 40], _stream())
    assert e.value.status == H.HDDM_EINVAL
    with pytest.raises(H.HddmError) as e:  # the same context twice
        H.hddm_apply_precond_batch([a.ctx, a.ctx], [256, 256], [1, 1], [256, 256], [1, 1], [1, 1],
                                   [256, 256], [1 << 40, 1 << 40], _stream())
    assert e.value.status == H.HDDM_EINVAL
    a.close()
    b.close()


def test_session_equals_block_solves_with_late_joins():
    """Three problems of different grids and media; the third joins after
    the first two have run 20 rounds.  Each finishes with the iteration
    counts, bitwise the solutions and the residual histories of its own
    hddm_solve_block."""
    import torch
    from paper_1508_02897_amd import hddm as H
    ws = [_workload(384, 1, 10.0), _workload(256, 5, 12.0), _workload(512, 2, 8.0)]
    nr = [2, 1, 3]
    restart = 3
    B = [np.stack([synth.gaussian_rhs(w.N, w.P, synth.gaussian_centers(w.N, 1, 70 * i + k))
                   for k in range(n)]) for i, (w, n) in enumerate(zip(ws, nr))]
    alone = []
    for w, b in zip(ws, B):
        s = _solver(w, restart)
        X, infos = s.solve_block(b, tol=1e-8, restart=restart, ortho=1)
        alone.append((X.cpu().numpy(), [i["iters"] for i in infos],
                      [s.history(k) for k in range(len(infos))]))
        s.close()
    ss = [_solver(w, restart) for w in ws]
    Bd = [torch.from_numpy(b).to("cuda") for b in B]
    Xd = [torch.empty_like(b) for b in Bd]
    bufs = [s.ensure_block(n, restart) for s, n in zip(ss, nr)]
    opts = H.SolveOpts(tol=1e-8, restart=restart, maxit=5000, ortho=1, reserved=0)
    sess = H.hddm_session_create()
    ids = {}

    def add(i):
        w = ws[i]
        wb, kb = bufs[i]
        ids[H.hddm_session_add(sess, ss[i].ctx, Bd[i].data_ptr(), w.Ng * w.Ng, Xd[i].data_ptr(),
                               w.Ng * w.Ng, nr[i], opts, wb.data_ptr(), wb.numel(),
                               kb.data_ptr(), kb.numel())] = i
    add(0)
    add(1)
    with pytest.raises(H.HddmError) as e:  # one problem per context
        add(1)
    assert e.value.status == H.HDDM_EINVAL
    infos, rounds = {}, 0
    while len(infos) < 3:
        if rounds == 20:
            add(2)
        for pid in H.hddm_session_step(sess, _stream()):
            infos[ids[pid]] = H.hddm_session_result(sess, pid, nr[ids[pid]])
        rounds += 1
        assert rounds < 5000
    H.hddm_session_destroy(sess)
    torch.cuda.synchronize()
    for i in range(3):
        X = Xd[i].cpu().numpy()
        its = [inf.iters for inf in infos[i]]
        print(f"session problem {i} ({ws[i].N}^2, {nr[i]} sources): iters {its} alone "
              f"{alone[i][1]}", flush=True)
        assert its == alone[i][1]
        assert all(inf.relres_true <= 1e-8 for inf in infos[i])
        assert np.array_equal(X, alone[i][0])
        # the convergence history of each session problem, kept on its context
        for k in range(nr[i]):
            assert np.array_equal(ss[i].history(k), alone[i][2][k])
    for s in ss:
        s.close()
