"""Serving loop on the GPU: requests of mixed sizes and media run concurrently
(own stream and context each, shared resident factors), every result reaches
the tolerance and matches the oracle's exact discrete solution, and each
result is identical whether the request ran in the mix or alone."""
import numpy as np
import pytest

from tests.gpu_common import gpu_ready

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a ROCm GPU")]


@pytest.mark.parametrize("mode,block_min_n", [("threads", 2048), ("threads", 256),
                                              ("batched", 0)])
def test_alone_vs_mix_identical_and_converged(mode, block_min_n):
    """threads: a host thread, stream and context per request (block_min_n =
    256: requests with several sources take the block form); batched: one
    solver session, every round one fused launch for all in-flight requests
    (box budget 20 boxes: a 512^2 request (16 boxes) runs with at most one
    256^2 request (4 boxes), so the loop also waits for box slots)."""
    from paper_1508_02897_amd.serving import BatchedServer, Server, make_requests
    reqs = make_requests(10, [256, 512], seed=11)
    cls = BatchedServer if mode == "batched" else Server
    extra = dict(box_budget=20) if mode == "batched" else dict(block_min_n=block_min_n)
    mix = cls(hbm_budget=40e9, max_inflight=4, keep_solutions=True, **extra)
    summary = mix.run(reqs)
    print(summary)
    assert summary["max_relres"] <= 1e-8
    assert summary["p99_latency_s"] >= summary["p50_latency_s"] > 0
    # the factor cache is reused: fewer factorisations than requests
    media = {(r.medium_seed, r.N) for r in reqs}
    assert summary["factorisations"] == len(media)
    # served solutions against the oracle's exact discrete solution (sparse
    # LU of the global PML system), one request per (medium, N)
    from oracle import Problem, direct
    from paper_1508_02897_amd.serving import medium_workload, request_rhs
    seen = set()
    for r in reqs:
        if (r.medium_seed, r.N) in seen:
            continue
        seen.add((r.medium_seed, r.N))
        w = medium_workload(r.N, r.medium_seed)
        prob = Problem.from_workload(w)
        for k, f in enumerate(request_rhs(r, w)[:1]):
            u = direct.sparse_solve(prob, f)
            d = np.linalg.norm(r.solutions[k] - u) / np.linalg.norm(u)
            print(r.rid, r.N, r.medium_seed, "source", k, "served vs oracle direct", d)
            assert d <= 1e-6
    for r in reqs[:8]:  # eight requests re-run alone
        alone = make_requests(10, [256, 512], seed=11)[r.rid]
        srv = cls(hbm_budget=40e9, max_inflight=1, keep_solutions=True, **extra)
        srv.run([alone])
        assert alone.iters == r.iters
        for a, b in zip(alone.solutions, r.solutions):
            d = np.linalg.norm(a - b) / np.linalg.norm(b)
            print(r.rid, r.N, r.medium_seed, "alone vs mix", d)
            assert d <= 1e-12


@pytest.mark.parametrize("mode", ["threads", "batched"])
def test_admission_waits_for_memory_then_evicts(mode):
    """A budget that holds one medium at a time still serves every request:
    later requests wait for memory and idle factors are evicted."""
    from paper_1508_02897_amd.serving import BatchedServer, Server, make_requests
    reqs = make_requests(6, [512], seed=3)
    cls = BatchedServer if mode == "batched" else Server
    srv = cls(hbm_budget=1.6e9 if mode == "threads" else 2.2e9, max_inflight=4, restart=10)
    summary = srv.run(reqs)
    print(summary)
    assert summary["requests"] == 6 and summary["max_relres"] <= 1e-8
    assert srv.used <= srv.budget


def test_batched_alone_vs_mix_larger_grids():
    """The batched loop at 1024^2 and 2048^2 (64 and 256 boxes per request,
    up to four requests and 1024 boxes in one fused sweep): every result
    converges and is bitwise the request's own result when served alone."""
    from paper_1508_02897_amd.serving import BatchedServer, make_requests
    reqs = make_requests(4, [1024, 2048], seed=13)
    mix = BatchedServer(hbm_budget=120e9, max_inflight=4, keep_solutions=True)
    summary = mix.run(reqs)
    print(summary, [(r.N, r.n_sources, min(r.iters), max(r.iters)) for r in reqs])
    assert summary["max_relres"] <= 1e-8
    for r in reqs:
        alone = make_requests(4, [1024, 2048], seed=13)[r.rid]
        BatchedServer(hbm_budget=120e9, max_inflight=1, keep_solutions=True).run([alone])
        print(r.rid, r.N, r.medium_seed, "iterations mix", r.iters, "alone", alone.iters)
        assert alone.iters == r.iters
        for a, b in zip(alone.solutions, r.solutions):
            assert np.array_equal(a, b)


def test_batched_sessions_per_size_class():
    """Requests split over two sessions by box count (here 512^2 requests,
    16 boxes, in a session of their own beside the 256^2 ones), each session
    on its own stream and host driver sharing the memory budget and the
    factor cache: every result converges and is bitwise the request's own
    result served alone."""
    from paper_1508_02897_amd.serving import BatchedServer, make_requests
    reqs = make_requests(8, [256, 512], seed=17)
    mix = BatchedServer(hbm_budget=40e9, max_inflight=4, keep_solutions=True, split_boxes=16)
    summary = mix.run(reqs)
    print(summary, [(r.N, r.n_sources, min(r.iters), max(r.iters)) for r in reqs])
    assert summary["max_relres"] <= 1e-8 and summary["split_boxes"] == 16
    assert {r.N for r in reqs} == {256, 512}
    media = {(r.medium_seed, r.N) for r in reqs}
    assert summary["factorisations"] == len(media)
    for r in reqs:
        alone = make_requests(8, [256, 512], seed=17)[r.rid]
        BatchedServer(hbm_budget=40e9, max_inflight=1, keep_solutions=True, split_boxes=0).run(
            [alone])
        assert alone.iters == r.iters
        for a, b in zip(alone.solutions, r.solutions):
            assert np.array_equal(a, b)


def test_batched_coalesces_requests_on_one_factor():
    """Requests that arrive together on the same medium and grid become one
    block problem (up to 16 sources): fewer problems than requests, and every
    request's iterations and solutions bitwise those it gets as a problem of
    its own."""
    from paper_1508_02897_amd.serving import BatchedServer, make_requests
    reqs = make_requests(12, [256], seed=19)
    media = {}
    for r in reqs:
        media.setdefault(r.medium_seed, []).append(r.n_sources)
    print({k: v for k, v in media.items()})
    assert any(len(v) > 1 and sum(v[:2]) <= 16 for v in media.values())
    srv = BatchedServer(hbm_budget=40e9, max_inflight=8, keep_solutions=True)
    summary = srv.run(reqs)
    print(summary)
    assert summary["coalesce"] and summary["problems"] < len(reqs)
    assert summary["max_relres"] <= 1e-8
    own = make_requests(12, [256], seed=19)
    s2 = BatchedServer(hbm_budget=40e9, max_inflight=8, keep_solutions=True, coalesce=False)
    summary2 = s2.run(own)
    assert summary2["problems"] == len(own)
    for a, b in zip(reqs, own):
        assert a.rid == b.rid and a.iters == b.iters
        for x, y in zip(a.solutions, b.solutions):
            assert np.array_equal(x, y)
