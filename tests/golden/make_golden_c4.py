"""Writes c4_4096_oracle.json: the oracle's DDM-preconditioned GMRES on the
4096^2 workload (4128^2 unknowns, 32x32 boxes of 168/176, random medium with
correlation length 40h, seed 4; right-hand side k is one Gaussian, seed
4000 + k).  Calls only `oracle` and `synth`.

A global direct solve does not fit a host at this size, so for each chosen
right-hand side the script records
  * the iteration count of GMRES(3) (the restart of the benchmark's block
    form) from x0 = 0 to relative residual 1e-8, with its true residual;
  * a reference solution: the same iteration continued from that iterate
    (restart 5) to relative residual 1e-10; its norm and its values at 4000
    seeded nodes;
  * the relative L2 distance of the 1e-8 iterate from the reference;
  * the residual estimate |gamma_{j+1}| / |b| after every Arnoldi step of
    the GMRES(3) run to 1e-8 ("history");
  * the oracle's times on this host (operator assembly, local factors, one
    application, the batched time to 1e-8) and the number of worker
    processes.
A right-hand side whose reference has not been computed yet is recorded
with its iteration count only ("partial"); a later run completes it.
The operator is the oracle's assembled sparse M (`oracle.operator.global_matrix`).
Local factors: SuperLU with the low-fill options (`oracle.ddm.LOW_FILL`),
about 30 GB for the 1024 boxes, spread over a process pool
(`oracle.pool.PooledOneStepDDM`, bitwise equal to the serial form factored
with one BLAS thread).

The chosen right-hand sides run side by side, one `oracle.gmres.gmres` call
per thread; their preconditioner applications meet in one pooled application
(`apply_many`: each local factor solves all their local sources at once, each
result bitwise the single application), so three right-hand sides cost little
more than one.  Each run is unchanged by this: it sees exactly the values a
run on its own with the same pool would see (a serial `ddm.OneStepDDM`
factored with a multi-threaded BLAS differs from the pool's one-thread
factors in the last bits only: relative 2e-15 in the iterate at 128^2, same
iteration counts).

The runs can be resumed: at the end of every few GMRES cycles each thread
stores its iterate and counts under the checkpoint folder (default: a folder
in the system's temporary directory), and a new start continues from there
(a restarted GMRES started again from the iterate of a cycle end takes the
same steps; pinned by a test).  The JSON file is rewritten after each
right-hand side finishes.

Run from the repository root:
    python tests/golden/make_golden_c4.py [rhs indices, default 0 7 15]
        [--workers W] [--checkpoint DIR] [--out JSON (default: beside this script)]
        [--history]
--history adds the history to records written before it was kept: only the
run to 1e-8 is repeated (the same steps), and the record's other values stay.
On a 16-core host with --workers 16: about 12 minutes for one right-hand
side (577 s to 1e-8, 130 s more for the reference), 16 minutes for two side
by side.  Hosts whose fresh memory pages are slow to map (some virtual
machines) take far longer.
"""
import json
import os
import sys
import tempfile
import threading
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import synth  # noqa: E402
from oracle import Problem, ddm, gmres, operator, pool  # noqa: E402

NAME = "c4_4096"
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{NAME}_oracle.json")
DESCRIPTION = ("4096^2 interior (4128^2 unknowns), P=16, 32x32 tiles of 128, n_ol=8, random medium "
               "corr 40h seed 4, 10 ppw at c=0.8; RHS k: 1 Gaussian seed 4000+k; GMRES(3) tol 1e-8, "
               "reference continued with GMRES(5) to 1e-10")
MAXIT = 5000
SAVE_EVERY = 8  # cycles between checkpoints


def keep_freed_memory():
    """Every GMRES step makes temporaries of the vector size (272 MB here);
    by default glibc maps each one afresh and unmaps it when freed, so every
    step pays the page faults of its temporaries again.  Serving all threads
    from the main heap (one arena), without separate mappings and without
    trimming, lets freed blocks be reused in place.  Does not change any
    value computed."""
    import ctypes
    try:
        libc = ctypes.CDLL("libc.so.6")
    except OSError:
        return
    M_TRIM_THRESHOLD, M_MMAP_MAX, M_ARENA_MAX = -1, -4, -8
    libc.mallopt(M_ARENA_MAX, 1)
    libc.mallopt(M_MMAP_MAX, 0)
    libc.mallopt(M_TRIM_THRESHOLD, 2 ** 31 - 1)


class Batcher:
    """Meets the preconditioner calls of the live GMRES threads: the last of
    them to arrive runs one pooled application for all and wakes the
    others.  A thread that has finished calls leave()."""

    def __init__(self, P, n):
        self.P = P
        self.live = n
        self.pending = {}
        self.results = {}
        self.round = 0
        self.cv = threading.Condition()
        self.rounds = 0

    def _run(self):
        ks = sorted(self.pending)
        zs = self.P.apply_many([self.pending[k] for k in ks])
        for k, z in zip(ks, zs):
            self.results[k] = z
        self.pending.clear()
        self.round += 1
        self.rounds += 1
        self.cv.notify_all()

    def apply(self, k, r):
        with self.cv:
            self.pending[k] = r
            mine = self.round
            if len(self.pending) == self.live:
                self._run()
            else:
                while self.round == mine:
                    self.cv.wait()
            return self.results.pop(k)

    def leave(self):
        with self.cv:
            self.live -= 1
            if self.pending and len(self.pending) == self.live:
                self._run()


def _save(path, **arrays):
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def main(argv):
    global PATH
    keep_freed_memory()
    workers = None
    history_only = "--history" in argv
    argv = [a for a in argv if a != "--history"]
    ckdir = os.path.join(tempfile.gettempdir(), f"{NAME}_oracle_checkpoints")
    for opt in ("--workers", "--checkpoint", "--out"):
        if opt in argv:
            i = argv.index(opt)
            if opt == "--workers":
                workers = int(argv[i + 1])
            elif opt == "--checkpoint":
                ckdir = argv[i + 1]
            else:
                PATH = argv[i + 1]
            argv = argv[:i] + argv[i + 2:]
    rhs_ids = [int(a) for a in argv] or [0, 7, 15]
    os.makedirs(ckdir, exist_ok=True)
    t0 = time.time()
    w = synth.config(NAME)
    prob = Problem.from_workload(w)
    M = operator.global_matrix(prob)  # the assembled operator, formed once
    t_setup = time.time() - t0
    print(f"operator assembled in {t_setup:.1f} s", flush=True)

    def A(u):
        return (M @ u.ravel()).reshape(u.shape)

    out = {"workload": DESCRIPTION, "rhs": {}}
    if os.path.exists(PATH):
        with open(PATH) as fh:
            out = json.load(fh)
    need = "history" if history_only else "samples"
    todo = [k for k in rhs_ids if need not in out["rhs"].get(str(k), {})]
    print(f"right-hand sides to run: {todo} (checkpoints in {ckdir})", flush=True)
    if not todo:
        return
    lock = threading.Lock()
    t0 = time.time()
    with pool.PooledOneStepDDM(prob, workers=workers, splu_options=ddm.LOW_FILL,
                               columns=len(todo)) as P:
        t_factor = time.time() - t0
        print(f"factors: {t_factor:.1f} s wall over {P.workers} workers", flush=True)
        r0 = synth.rhs_for(w, todo[0])
        t0 = time.time()
        P.apply(r0)
        t_apply = time.time() - t0
        print(f"one application: {t_apply:.2f} s", flush=True)
        batch = Batcher(P, len(todo))
        t_start = time.time()
        errors = []

        def run(k):
            try:
                _run_rhs(k)
            except BaseException as e:  # noqa: BLE001 - reported by the main thread
                errors.append((k, e))
                raise
            finally:
                batch.leave()

        def _run_rhs(k):
            f = synth.rhs_for(w, k)
            nb = np.linalg.norm(f)
            Pk = lambda r: batch.apply(k, r)  # noqa: E731
            done1 = os.path.join(ckdir, f"rhs{k}_1e-8.npz")
            spent = {}
            hist = []
            phases = ((1, w.tol, 3),) if history_only else ((1, w.tol, 3), (2, 1e-10, 5))
            for phase, tol, restart in phases:
                ck = os.path.join(ckdir, f"rhs{k}_phase{phase}.npz")
                if phase == 2:
                    d = np.load(done1)
                    x1 = d["x"]
                    info1 = {key: d[key].item() for key in ("iters", "restarts", "relres_true",
                                                            "seconds")}
                    hist = [float(v) for v in d["hist"]] if "hist" in d else []
                if phase == 1 and os.path.exists(done1) and not history_only:
                    continue
                x0, it0, cyc0, sec0 = (None, 0, 0, 0.0) if phase == 1 else (x1, 0, 0, 0.0)
                if os.path.exists(ck):
                    d = np.load(ck)
                    x0, it0, cyc0, sec0 = d["x"], int(d["iters"]), int(d["restarts"]), \
                        float(d["seconds"])
                    if phase == 1:
                        hist = [float(v) for v in d["hist"]] if "hist" in d else []
                    print(f"rhs {k} phase {phase}: resuming after {it0} iterations", flush=True)
                t1 = time.time()

                def cb(it, est):
                    if phase == 1:
                        hist.append(float(est))
                    if (it0 + it) % 25 == 0:
                        print(f"rhs {k} phase {phase} iter {it0 + it} est {est:.3e} "
                              f"({sec0 + time.time() - t1:.0f} s)", flush=True)

                def cyc(x, it, c):
                    if c % SAVE_EVERY == 0:
                        _save(ck, x=x, iters=it0 + it, restarts=cyc0 + c,
                              seconds=sec0 + time.time() - t1, hist=np.array(hist))

                x, info = gmres.gmres(A, Pk, f, tol=tol, restart=restart, maxit=MAXIT - it0,
                                      x0=x0, callback=cb, cycle_callback=cyc)
                iters, restarts = it0 + info["iters"], cyc0 + info["restarts"]
                seconds = sec0 + time.time() - t1
                spent[phase] = seconds
                if phase == 1:
                    _save(done1, x=x, iters=iters, restarts=restarts,
                          relres_true=info["relres_true"], seconds=seconds, hist=np.array(hist))
                    print(f"rhs {k}: {iters} iterations to {info['relres_true']:.3e} in "
                          f"{seconds:.0f} s", flush=True)
                    if history_only:
                        with lock:
                            rec = out["rhs"][str(k)]
                            if rec.get("iters") != int(iters):
                                print(f"rhs {k}: {iters} iterations now, {rec.get('iters')} "
                                      f"recorded", flush=True)
                            rec["history"] = hist
                            rec["history_run"] = {"iters": int(iters), "seconds": seconds,
                                                  "workers": P.workers,
                                                  "host_cpus": os.cpu_count()}
                            with open(PATH, "w") as fh:
                                json.dump(out, fh)
                        print(f"rhs {k}: history of {len(hist)} steps written", flush=True)
                        return
                    # the count first, in case the reference does not finish
                    with lock:
                        out["rhs"][str(k)] = {
                            "iters": int(iters), "restarts": int(restarts),
                            "relres_true": float(info["relres_true"]),
                            "history": hist,
                            "partial": "no reference solution yet",
                            "oracle_seconds": {"setup": t_setup, "factor_wall": t_factor,
                                               "one_apply": t_apply, "to_1e-8": seconds},
                            "batched_rhs": len(todo), "workers": P.workers,
                            "host_cpus": os.cpu_count()}
                        with open(PATH, "w") as fh:
                            json.dump(out, fh)
                else:
                    u, iters2 = x, iters
            rel_ref = float(np.linalg.norm(f - A(u)) / nb)
            print(f"rhs {k}: reference after {iters2} more iterations, relres {rel_ref:.3e}",
                  flush=True)
            rng = np.random.default_rng(12345 + k)
            iy = rng.integers(0, w.Ng, 4000)
            ix = rng.integers(0, w.Ng, 4000)
            rec = {
                "iters": int(info1["iters"]),
                "restarts": int(info1["restarts"]),
                "relres_true": float(info1["relres_true"]),
                "ref_relres": rel_ref,
                "ref_extra_iters": int(iters2),
                "x_1e8_vs_ref_relL2": float(np.linalg.norm(x1 - u) / np.linalg.norm(u)),
                "history": hist,
                "u_norm": float(np.linalg.norm(u)),
                "samples": [[int(a), int(b), float(u[a, b].real), float(u[a, b].imag)]
                            for a, b in zip(iy, ix)],
                "oracle_seconds": {"setup": t_setup, "factor_wall": t_factor, "one_apply": t_apply,
                                   "to_1e-8": float(info1["seconds"]),
                                   "reference": float(spent.get(2, 0.0))},
                "batched_rhs": len(todo),
                "workers": P.workers,
                "host_cpus": os.cpu_count(),
            }
            with lock:
                out["rhs"][str(k)] = rec
                with open(PATH, "w") as fh:
                    json.dump(out, fh)
            print(f"rhs {k} written", flush=True)

        threads = [threading.Thread(target=run, args=(k,)) for k in todo]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        print(f"all done in {time.time() - t_start:.0f} s, {batch.rounds} pooled applications",
              flush=True)
        if errors:
            raise RuntimeError(f"right-hand sides failed: {errors}")


if __name__ == "__main__":
    main(sys.argv[1:])
