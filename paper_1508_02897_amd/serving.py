"""Continuous-batching request loop over the C ABI.

Requests (grid size N, medium seed, 1-8 Gaussian sources) arrive over time.
The server:
  * keeps factorisations resident in an LRU cache keyed by (medium seed, N),
    so requests for a medium already seen skip the factor and reuse it for
    every right-hand side (the local factorisation is a one-time setup, Sec. 3);
  * admits an arrived request as soon as a slot is free and the HBM it needs
    fits the budget (default: 85% of the device memory free at start): its
    factor (if not resident) + a workspace lane + the Krylov bases; idle
    cached factors are evicted LRU-first to make room, and requests wait
    (first come, first served) when nothing can be evicted;
  * batched mode (BatchedServer, the default): solver sessions
    (hddm_session_*), each with a driver loop, a stream and a host thread of
    its own: the requests that fill the device by themselves (at least one
    box per SIMD: 4096^2 with tiles of 128) in one, all smaller ones in
    another, so small requests never queue behind a large one.  Every
    admitted request is one block FGMRES problem holding all its sources, on
    its own context that shares the resident factor (hddm_share_factor);
    every round advances all in-flight requests of a session with ONE fused
    preconditioner launch over the union of their boxes (the block sweep of
    up to 8 problems of different grids, media and wave numbers), then their
    Arnoldi steps and one wait.  Requests join between rounds while others
    iterate, as long as their boxes fit the session's box budget (one per
    SIMD: a round's sweep covers every box in one pass), and leave when all
    their sources converged.  Arrived requests on the same factor (same
    medium and N) are admitted together as one problem of up to 16 sources,
    so one block sweep reads each G_j once for all of them;
  * threads mode (Server): every admitted request runs on its own host
    thread and HIP stream with its own context, so kernels of different
    requests overlap through the hardware queues; a request's sources are
    solved together through the block form when that is faster than one after
    another (from 2048^2 with two or more sources, at 1024^2 with seven or
    more);
  * records latency = completion - arrival per request and reports p50/p99
    beside solves/s and right-hand sides/s.

Each result is independent of the mix: a request's kernels are deterministic
(fixed-order reductions, no atomics), read only the shared factor and write
only the request's own buffers; in batched mode each problem's iterates are
bitwise those of its own block solve.

Media: seeds 0-3 draw the random medium (correlation length 20h), seeds 4-7
the three-layer medium; each seed fixes its points per wavelength,
(8, 10, 12)[seed % 3], so a medium and its factorisation can be reused.

    python -m paper_1508_02897_amd.serving --requests 60 --sizes 512,1024
    python -m paper_1508_02897_amd.serving --requests 200 --closed-only
    python -m paper_1508_02897_amd.serving --requests 200 --rate 0.298 [--mode threads]
"""
import argparse
import json
import os
import sys
import threading
import time
from dataclasses import dataclass, field, replace

import numpy as np

from . import hddm as H

PPW = (8.0, 10.0, 12.0)


@dataclass
class Request:
    rid: int
    N: int
    medium_seed: int
    n_sources: int
    source_seed: int
    arrival: float = 0.0
    # filled by the server
    start: float = -1.0
    done: float = -1.0
    iters: list = field(default_factory=list)
    relres: list = field(default_factory=list)
    factored_here: bool = False
    solutions: list = None


def medium_workload(N, seed, tile=128, n_ol=8, P=16):
    """Workload record of a serving medium (grid N, seed-fixed generator/ppw)."""
    import synth
    kind = "random" if seed < 4 else "layered"
    c_min = 0.8 if kind == "random" else 1.0
    return synth.Workload(name=f"serve_{kind}_{seed}_{N}", N=N, P=P, tile=tile, n_ol=n_ol,
                          ppw=PPW[seed % 3], c_min=c_min, medium=kind, medium_seed=seed,
                          corr_len_h=20.0)


def make_requests(n, sizes, seed=5, rate=None):
    """n requests with N uniform in `sizes`, medium seed uniform in 0..7, 1-8
    sources; Poisson arrivals at `rate` per second (all at t=0 if None).  The
    requests themselves do not depend on `rate` (arrival times come from a
    second generator), so a closed-loop and an open-loop pass serve the same
    requests."""
    rng = np.random.default_rng(seed)
    out = [Request(rid=i, N=int(rng.choice(sizes)), medium_seed=int(rng.integers(0, 8)),
                   n_sources=int(rng.integers(1, 9)), source_seed=100000 + i)
           for i in range(n)]
    if rate:
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, n)
        for r, t in zip(out, np.cumsum(gaps)):
            r.arrival = float(t)
    return out


def request_rhs(req, w):
    """Right-hand sides of a request: source s is one Gaussian from seed
    source_seed * 16 + s."""
    import synth
    return [synth.gaussian_rhs(w.N, w.P, synth.gaussian_centers(w.N, 1, req.source_seed * 16 + s))
            for s in range(req.n_sources)]


def coalesce_group(pending, i, now, taken, max_sources):
    """The requests that share one block problem with pending[i]: itself,
    then, in arrival order, every later request that has arrived by `now`,
    is not already `taken`, has the same grid and medium (so the same
    factor), and still fits `max_sources` sources in all."""
    lead = pending[i]
    group, total = [lead], lead.n_sources
    for r in pending[i + 1:]:
        if r.arrival > now:
            break
        if (r.rid not in taken and r.N == lead.N and r.medium_seed == lead.medium_seed
                and total + r.n_sources <= max_sources):
            group.append(r)
            total += r.n_sources
    return group


def _with_retry(torch, fn):
    """fn() once more after returning the caching allocator's free blocks to
    the device, if the first attempt ran out of memory (blocks freed by
    earlier requests can be cached in sizes no longer asked for)."""
    try:
        return fn()
    except torch.OutOfMemoryError:
        torch.cuda.empty_cache()
        return fn()


class _Medium:
    def __init__(self, key, w):
        self.key = key
        self.w = w
        self.base = None          # Solver owning the factor buffer
        self.ready = threading.Event()
        self.error = None
        self.lanes = []           # idle Solvers sharing the factor
        self.users = 0
        self.last_used = 0.0
        self.velocity = None


class Server:
    def __init__(self, hbm_budget=None, max_inflight=8, restart=3, tol=1e-8, maxit=20000,
                 device=0, keep_solutions=False, block=True, block_min_n=2048, progress=False,
                 box_budget=None):
        """hbm_budget: device bytes the server may hold (factors, lanes,
        Krylov bases); default 85% of the device memory free at start.
        box_budget (batched mode): boxes of the problems iterating together in
        one session (see BatchedServer)."""
        import torch
        self.torch = torch
        self.device = device
        if hbm_budget is None:
            hbm_budget = 0.85 * torch.cuda.mem_get_info(device)[0]
        self.budget = float(hbm_budget)
        if box_budget is None:
            box_budget = 4 * torch.cuda.get_device_properties(device).multi_processor_count
        self.box_budget = int(box_budget)
        self.max_inflight = max_inflight
        self.restart = restart
        self.tol = tol
        self.maxit = maxit
        self.keep_solutions = keep_solutions
        self.block = block
        self.block_min_n = block_min_n
        self.progress = progress
        self.media = {}
        self._size_cache = {}
        self.used = 0.0
        self.lock = threading.Condition()

    # -- memory accounting -------------------------------------------------
    def use_block(self, N, n_sources):
        """Whether a request's sources are solved together (see the module doc;
        block_min_n = 2048 by default)."""
        return self.block and n_sources >= 2 and (
            N >= self.block_min_n or (N >= self.block_min_n // 2 and n_sources >= 7))

    def _sizes(self, w):
        """(factor bytes, work bytes, Krylov bytes per right-hand side, block
        workspace bytes) for grid N (medium-independent)."""
        if w.N not in self._size_cache:
            from .solver import problem_from_workload
            ctx = H.hddm_setup(problem_from_workload(w, H.HDDM_MIXED_C64),
                               np.ones((w.Ng, w.Ng)), self.device)
            try:
                fb, wb, kb = H.hddm_query_bytes(ctx, self.restart)
                bw, bk = H.hddm_query_block_bytes(ctx, 2, self.restart)
            finally:
                H.hddm_destroy(ctx)
            self._size_cache[w.N] = (float(fb), float(wb), float(kb), float(bw))
        return self._size_cache[w.N]

    def _lane_bytes(self, w, n_sources):
        """Device bytes a request's lane holds: workspace + one Krylov region
        (single form) and, in the block form, one region per source + the block
        workspace, so a block lane can later serve a single-source request
        without allocating more."""
        fb, wb, kb, bw = self._sizes(w)
        if self.use_block(w.N, n_sources):
            return wb + (n_sources + 1) * kb + bw
        return wb + kb

    def _evict_for(self, need, keep):
        """Evict idle media (LRU), never `keep`, until `need` more bytes fit.
        Called with the lock held."""
        idle = sorted((m for m in self.media.values()
                       if m.users == 0 and m.ready.is_set() and m.key != keep),
                      key=lambda m: m.last_used)
        for m in idle:
            if self.used + need <= self.budget:
                break
            fb = self._sizes(m.w)[0]
            self.used -= fb + sum(ln.lane_bytes for ln in m.lanes)
            for ln in m.lanes:
                ln.close()
            if m.base is not None:
                m.base.close()
            m.lanes, m.base = [], None
            del self.media[m.key]
        # then idle lanes of the kept medium itself (its factor stays)
        km = self.media.get(keep)
        if km is not None and self.used + need > self.budget:
            for ln in sorted(km.lanes, key=lambda ln: ln.lane_bytes):
                if self.used + need <= self.budget:
                    break
                if ln is km.base:
                    continue
                self.used -= ln.lane_bytes
                ln.close()
                km.lanes.remove(ln)
        if self.used + need <= self.budget:
            self.torch.cuda.empty_cache()
            return True
        return False

    # -- one request -------------------------------------------------------
    def _serve(self, req, m, lane, creator, lane_b, t0):
        from .solver import Solver, problem_from_workload
        import synth
        torch = self.torch
        w = m.w
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(stream):
            if creator:
                try:
                    m.velocity = synth.medium_for(w)
                    m.base = Solver(problem_from_workload(w, H.HDDM_MIXED_C64), m.velocity,
                                    device=self.device, restart=self.restart)
                    m.base.factor()
                    stream.synchronize()
                    req.factored_here = True
                except Exception as e:  # surfaced by run()
                    m.error = e
                m.ready.set()
            m.ready.wait()
            if m.error is not None:
                raise m.error
            if lane is None and creator:
                lane = m.base  # the factor owner is the creator's lane
            elif lane is None:
                lane = Solver(problem_from_workload(w, H.HDDM_MIXED_C64), m.velocity,
                              device=self.device, restart=self.restart, share_from=m.base)
            lane.lane_bytes = lane_b
            sols = []
            F = request_rhs(req, w)
            if self.use_block(w.N, len(F)):
                X, infos = lane.solve_block(np.stack(F), tol=self.tol, restart=self.restart,
                                            maxit=self.maxit)
                req.iters.extend(i["iters"] for i in infos)
                req.relres.extend(i["relres_true"] for i in infos)
                if self.keep_solutions:
                    sols = [x.cpu().numpy() for x in X]
            else:
                for f in F:
                    x, info = lane.solve(f, tol=self.tol, restart=self.restart, maxit=self.maxit)
                    req.iters.append(info["iters"])
                    req.relres.append(info["relres_true"])
                    if self.keep_solutions:
                        sols.append(x.cpu().numpy())
            stream.synchronize()
        req.solutions = sols if self.keep_solutions else None
        with self.lock:
            m.lanes.append(lane)
            m.users -= 1
            m.last_used = time.perf_counter()
            req.done = time.perf_counter() - t0
            self.inflight -= 1
            if self.progress:  # under the lock, so lines of concurrent requests do not mix
                print(f"# request {req.rid}: N={req.N} medium {req.medium_seed} sources "
                      f"{req.n_sources} latency {req.done - req.arrival:.2f} s iterations "
                      f"{min(req.iters)}-{max(req.iters)}", flush=True)
            self.lock.notify_all()

    def _admit(self, req):
        """Reserve what `req` needs; returns (medium, idle lane or None, creator,
        lane bytes) or None if it does not fit yet.  An idle lane is reused
        only if it holds at least what the request needs.  Called with the
        lock held."""
        w = medium_workload(req.N, req.medium_seed)
        key = (req.medium_seed, req.N)
        fb = self._sizes(w)[0]
        lane_b = self._lane_bytes(w, req.n_sources)
        m = self.media.get(key)
        lane = None
        if m is not None:
            fits = [ln for ln in m.lanes if ln.lane_bytes >= lane_b]
            if fits:
                lane = min(fits, key=lambda ln: ln.lane_bytes)
                m.lanes.remove(lane)
                lane_b = lane.lane_bytes
        need = (fb if m is None else 0.0) + (lane_b if lane is None else 0.0)
        if self.used + need > self.budget and not self._evict_for(need, key):
            if lane is not None:
                m.lanes.append(lane)
            return None
        self.used += need
        creator = m is None
        if creator:
            m = _Medium(key, w)
            self.media[key] = m
        m.users += 1
        return m, lane, creator, lane_b

    # -- the loop ------------------------------------------------------------
    def run(self, requests):
        """Serve `requests` (arrival times relative to the start); returns a
        summary dict.  Blocks until every request is done."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        self.inflight = 0
        threads, errors = [], []
        t0 = time.perf_counter()

        def worker(req, m, lane, creator, lane_b):
            try:
                self._serve(req, m, lane, creator, lane_b, t0)
            except Exception as e:  # keep the loop alive; report at the end
                errors.append((req.rid, repr(e)))
                with self.lock:
                    m.users -= 1
                    self.inflight -= 1
                    self.lock.notify_all()

        i = 0
        with self.lock:
            while i < len(pending) or self.inflight > 0:
                now = time.perf_counter() - t0
                started = False
                if i < len(pending) and pending[i].arrival <= now and self.inflight < self.max_inflight:
                    req = pending[i]
                    got = self._admit(req)
                    if got is not None:
                        req.start = now
                        self.inflight += 1
                        th = threading.Thread(target=worker, args=(req, *got), daemon=True)
                        threads.append(th)
                        th.start()
                        i += 1
                        started = True
                    elif self.inflight == 0:
                        raise RuntimeError(f"request {req.rid} does not fit the "
                                           f"{self.budget / 1e9:.1f} GB budget")
                if not started:
                    wait = 0.05
                    if i < len(pending) and pending[i].arrival > now:
                        wait = min(wait, pending[i].arrival - now)
                    self.lock.wait(timeout=max(wait, 1e-3))
        for th in threads:
            th.join()
        if errors:
            raise RuntimeError(f"requests failed: {errors[:3]}")
        makespan = time.perf_counter() - t0
        lat = np.array([r.done - r.arrival for r in requests])
        n_rhs = sum(r.n_sources for r in requests)
        return {
            "requests": len(requests),
            "rhs": n_rhs,
            "makespan_s": makespan,
            "solves_per_s": len(requests) / makespan,
            "rhs_per_s": n_rhs / makespan,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "max_latency_s": float(lat.max()),
            "factorisations": sum(1 for r in requests if r.factored_here),
            "max_relres": max(max(r.relres) for r in requests),
        }


class BatchedServer(Server):
    """The same requests, media cache and admission by HBM bytes, served
    through solver sessions (hddm_session_*): every admitted request is one
    block FGMRES problem (all its sources), and every round advances all
    problems of a session with one fused preconditioner launch over the
    union of their boxes (one block sweep for up to 8 problems of different
    grids, media and wave numbers), then their Arnoldi steps.  Requests join
    a session between rounds as soon as they have arrived, fit the HBM
    budget, a problem slot is free (8) and their boxes fit the box budget;
    they leave when all their sources have converged.  Requests of at least
    `split_boxes` boxes go to a session of their own, driven by its own host
    thread on its own stream, so that their rounds (which take every SIMD)
    and those of the smaller requests interleave on the device (measured on
    the 200-request workload at 0.298 requests/s: p50 1.9 s, p99 73.7 s,
    against p50 18.5 s / 10.6 s with one session at one / two boxes per
    SIMD, the same throughput).  With `coalesce` (the default), a request
    admitted while later-arrived requests on the same factor wait takes them
    along: their sources become the columns of one block problem (up to 16),
    so each round reads the factor once for all of them; each request is
    done when the problem is.  Each result is bitwise the request's own block
    solve (every column's arithmetic is independent of the other columns, and
    the session keeps each problem's iterates), so it is the same alone and
    in the mix, whatever the sessions and whichever requests share its
    problem."""

    def _lane_bytes(self, w, n_sources):
        fb, wb, kb, bw = self._sizes(w)
        # workspace, one Krylov region per source + summaries, block workspace,
        # and the request's right-hand sides and solutions (complex128)
        return wb + (n_sources + 1) * kb + bw + 2 * n_sources * 16.0 * w.Ng * w.Ng

    def __init__(self, *args, split_boxes=-1, coalesce=True, **kw):
        """split_boxes: requests with at least this many boxes iterate in a
        session of their own, on a stream and host driver of their own, so
        the others never wait behind them (default -1: the SIMD count, i.e.
        the 4096^2 requests of 128-node tiles; 0: one session for all).  The
        box budget (default: the SIMD count per session when split, twice it
        for a single session) caps each session's boxes.  coalesce: admit
        arrived requests on the same factor together as one problem."""
        box_budget = kw.pop("box_budget", None)
        self.coalesce = bool(coalesce)
        super().__init__(*args, box_budget=box_budget, **kw)
        simds = 4 * self.torch.cuda.get_device_properties(self.device).multi_processor_count
        self.split_boxes = simds if split_boxes == -1 else int(split_boxes)
        if box_budget is None:
            self.box_budget = simds if self.split_boxes else 2 * simds

    def run(self, requests):
        torch = self.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        self.problems = 0
        t0 = time.perf_counter()
        nbox = lambda r: (r.N // 128) ** 2  # noqa: E731
        if self.split_boxes:
            classes = [[r for r in pending if nbox(r) < self.split_boxes],
                       [r for r in pending if nbox(r) >= self.split_boxes]]
        else:
            classes = [pending]
        classes = [c for c in classes if c]
        errors = []

        def drive(sub):
            try:
                with torch.cuda.stream(torch.cuda.Stream(device=self.device)):
                    self._drive(sub, t0)
            except BaseException as e:  # noqa: BLE001 - re-raised below
                errors.append(e)

        if len(classes) == 1:
            drive(classes[0])
        else:
            threads = [threading.Thread(target=drive, args=(c,), daemon=True) for c in classes]
            for th in threads:
                th.start()
            for th in threads:
                th.join()
        if errors:
            raise errors[0]
        torch.cuda.synchronize()
        makespan = time.perf_counter() - t0
        lat = np.array([r.done - r.arrival for r in requests])
        n_rhs = sum(r.n_sources for r in requests)
        return {
            "mode": "batched",
            "requests": len(requests),
            "rhs": n_rhs,
            "makespan_s": makespan,
            "solves_per_s": len(requests) / makespan,
            "rhs_per_s": n_rhs / makespan,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "max_latency_s": float(lat.max()),
            "factorisations": sum(1 for r in requests if r.factored_here),
            "max_relres": max(max(r.relres) for r in requests),
            "box_budget": self.box_budget,
            "split_boxes": self.split_boxes,
            "coalesce": self.coalesce,
            "problems": self.problems,
        }

    def _drive(self, pending, t0):
        """One session serving `pending` (sorted by arrival) on the current
        stream: admission between rounds, one fused round per step."""
        from .solver import Solver, problem_from_workload
        import synth
        torch = self.torch
        stream = torch.cuda.current_stream(self.device).cuda_stream
        opts = H.SolveOpts(tol=self.tol, restart=self.restart, maxit=self.maxit,
                           ortho=H.ORTHO_CGS2_GRAM, reserved=0)
        sess = H.hddm_session_create()
        active = {}  # session id -> (requests, medium, lane, B, X, boxes)
        taken = set()  # rids admitted early, with the problem of an earlier request
        boxes_used = 0
        i = 0
        try:
            while i < len(pending) or active:
                now = time.perf_counter() - t0
                # admit arrived requests in order while they fit
                while (i < len(pending) and pending[i].arrival <= now
                       and len(active) < min(H.HDDM_BATCH_MAX, self.max_inflight)):
                    req = pending[i]
                    if req.rid in taken:
                        i += 1
                        continue
                    nbox = (req.N // 128) ** 2
                    if active and boxes_used + nbox > self.box_budget:
                        break
                    # arrived requests on the same factor join this one's problem
                    group = (coalesce_group(pending, i, now, taken, H.HDDM_BLOCK_MAX)
                             if self.coalesce else [req])
                    total = sum(r.n_sources for r in group)
                    with self.lock:
                        got = self._admit(req if len(group) == 1
                                          else replace(req, n_sources=total))
                    if got is None:
                        if not active:
                            with self.lock:  # the other session may still release memory
                                busy = any(m.users for m in self.media.values())
                            if busy:
                                time.sleep(0.01)
                                break
                            raise RuntimeError(f"request {req.rid} does not fit the "
                                               f"{self.budget / 1e9:.1f} GB budget")
                        break
                    m, lane, creator, lane_b = got
                    w = m.w
                    if creator:
                        m.velocity = synth.medium_for(w)
                        m.base = _with_retry(torch, lambda: Solver(
                            problem_from_workload(w, H.HDDM_MIXED_C64), m.velocity,
                            device=self.device, restart=self.restart))
                        m.base.factor()
                        m.ready.set()  # evictable once idle
                        req.factored_here = True
                        lane = m.base
                    elif lane is None:
                        lane = _with_retry(torch, lambda: Solver(
                            problem_from_workload(w, H.HDDM_MIXED_C64), m.velocity,
                            device=self.device, restart=self.restart, share_from=m.base))
                    lane.lane_bytes = lane_b
                    F = np.stack([f for r in group for f in request_rhs(r, w)])
                    B = _with_retry(torch, lambda: torch.from_numpy(F).to(lane.device))
                    X = _with_retry(torch, lambda: torch.empty_like(B))
                    wb, kb = _with_retry(torch, lambda: lane.ensure_block(total, self.restart))
                    n = w.Ng * w.Ng
                    pid = H.hddm_session_add(sess, lane.ctx, B.data_ptr(), n, X.data_ptr(), n,
                                             total, opts, wb.data_ptr(), wb.numel(),
                                             kb.data_ptr(), kb.numel())
                    start = time.perf_counter() - t0
                    for r in group:
                        r.start = start
                    taken.update(r.rid for r in group[1:])
                    active[pid] = (group, m, lane, B, X, nbox)
                    with self.lock:
                        self.problems += 1
                    boxes_used += nbox
                    i += 1
                if not active:
                    if i < len(pending):
                        time.sleep(max(0.001, min(0.05, pending[i].arrival - now)))
                    continue
                for pid in H.hddm_session_step(sess, stream):
                    group, m, lane, B, X, nbox = active.pop(pid)
                    total = sum(r.n_sources for r in group)
                    infos = H.hddm_session_result(sess, pid, total, raise_on_noconv=False)
                    sols = X.cpu().numpy() if self.keep_solutions else None
                    done = time.perf_counter() - t0
                    k = 0
                    for r in group:  # the problem's columns, request by request
                        part = slice(k, k + r.n_sources)
                        k += r.n_sources
                        r.iters = [inf.iters for inf in infos[part]]
                        r.relres = [inf.relres_true for inf in infos[part]]
                        if self.keep_solutions:
                            r.solutions = list(sols[part])
                        r.done = done
                    boxes_used -= nbox
                    with self.lock:
                        m.lanes.append(lane)
                        m.users -= 1
                        m.last_used = time.perf_counter()
                        if self.progress:  # under the lock: lines of the sessions do not mix
                            tag = f" (one problem with {len(group) - 1} more)" if len(group) > 1 else ""
                            for r in group:
                                print(f"# request {r.rid}: N={r.N} medium {r.medium_seed} "
                                      f"sources {r.n_sources} latency {r.done - r.arrival:.2f}"
                                      f" s iterations {min(r.iters)}-{max(r.iters)}{tag}",
                                      flush=True)
                    del B, X
        finally:
            H.hddm_session_destroy(sess)
        torch.cuda.current_stream(self.device).synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--sizes", default="512,1024,2048,4096")
    ap.add_argument("--budget-gb", type=float, default=None,
                    help="device memory the server may hold (default: 85%% of the free HBM)")
    ap.add_argument("--mode", default="batched", choices=["batched", "threads"],
                    help="batched: one driver, one fused launch per round for all in-flight "
                         "requests (solver session); threads: a host thread, stream and "
                         "context per request")
    ap.add_argument("--max-inflight", type=int, default=8)
    ap.add_argument("--box-budget", type=int, default=None,
                    help="batched mode: boxes of the requests iterating together in one session "
                         "(default: one per SIMD, twice that with --split-boxes 0)")
    ap.add_argument("--split-boxes", type=int, default=-1,
                    help="batched mode: requests with at least this many boxes get a session of "
                         "their own (default: the SIMD count; 0: one session for all)")
    ap.add_argument("--no-coalesce", action="store_true",
                    help="batched mode: one problem per request, even when arrived requests "
                         "share a factor")
    ap.add_argument("--restart", type=int, default=3)
    ap.add_argument("--load", type=float, default=0.8,
                    help="arrival rate as a fraction of the measured closed-loop capacity")
    ap.add_argument("--closed-only", action="store_true",
                    help="measure the closed-loop capacity only")
    ap.add_argument("--rate", type=float, default=None,
                    help="serve the open-loop pass at this arrival rate (requests/s) without "
                         "a closed-loop pass first")
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--quiet", action="store_true", help="no per-request progress lines")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sizes = [int(s) for s in args.sizes.split(",")]
    cls = BatchedServer if args.mode == "batched" else Server
    extra = (dict(box_budget=args.box_budget, split_boxes=args.split_boxes,
                  coalesce=not args.no_coalesce)
             if args.mode == "batched" else {})
    srv = cls(hbm_budget=None if args.budget_gb is None else args.budget_gb * 1e9,
              max_inflight=args.max_inflight, restart=args.restart, progress=not args.quiet,
              **extra)
    closed = None
    if args.rate is None:
        # closed loop (every request at t = 0) -> capacity
        closed = srv.run(make_requests(args.requests, sizes, seed=args.seed))
        closed["sizes"] = sizes
        closed["restart"] = args.restart
        print("# closed loop:", json.dumps(closed), flush=True)
        if args.closed_only:
            return
        rate = args.load * closed["solves_per_s"]
    else:
        rate = args.rate
    reqs = make_requests(args.requests, sizes, seed=args.seed, rate=rate)
    open_ = srv.run(reqs)
    open_["arrival_rate_per_s"] = rate
    open_["sizes"] = sizes
    open_["restart"] = args.restart
    if closed is not None:
        open_["load"] = args.load
        open_["closed_loop_solves_per_s"] = closed["solves_per_s"]
        open_["note"] = ("p99 of this many samples is a high order statistic and noisy; "
                         "factor cache warm from the closed-loop pass")
    else:
        open_["note"] = ("arrival rate given on the command line; factor cache cold at the "
                         "start; p99 of this many samples is a high order statistic")
    print(json.dumps(open_), flush=True)


if __name__ == "__main__":
    main()
