"""Writes c4_4096_oracle.json: the oracle's DDM-preconditioned GMRES on the
4096^2 workload (4128^2 unknowns, 32x32 boxes of 168/176, random medium with
correlation length 40h, seed 4; right-hand side k is one Gaussian, seed
4000 + k).  Calls only `oracle` and `synth`.

A global direct solve does not fit a host at this size, so for each chosen
right-hand side the script records
  * the iteration count of GMRES(3) (the restart of the benchmark's block
    form) from x0 = 0 to relative residual 1e-8, with its true residual;
  * a reference solution: the same iteration continued from that iterate
    (restart 10) to relative residual 1e-10; its norm and its values at 4000
    seeded nodes;
  * the relative L2 distance of the 1e-8 iterate from the reference;
  * the oracle's times on this host (local factors, one application, time to
    1e-8) and the number of worker processes.
The operator is the oracle's assembled sparse M (`oracle.operator.global_matrix`).
Local factors: SuperLU with the low-fill options (`oracle.ddm.LOW_FILL`),
about 30 GB for the 1024 boxes, spread over a process pool
(`oracle.pool.PooledOneStepDDM`, bitwise equal to the serial form).
The file is rewritten after each right-hand side.

Run from the repository root:
    python tests/golden/make_golden_c4.py [rhs indices, default 0 7 15] [--workers W]
Takes about 40 minutes per right-hand side on 8 cores.
"""
import json
import os
import sys
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
               "reference continued with GMRES(10) to 1e-10")


def main(argv):
    workers = None
    if "--workers" in argv:
        i = argv.index("--workers")
        workers = int(argv[i + 1])
        argv = argv[:i] + argv[i + 2:]
    rhs_ids = [int(a) for a in argv] or [0, 7, 15]
    w = synth.config(NAME)
    prob = Problem.from_workload(w)
    M = operator.global_matrix(prob)  # the assembled operator, formed once

    def A(u):
        return (M @ u.ravel()).reshape(u.shape)

    out = {"workload": DESCRIPTION, "rhs": {}}
    if os.path.exists(PATH):
        with open(PATH) as fh:
            out = json.load(fh)
    t0 = time.time()
    with pool.PooledOneStepDDM(prob, workers=workers, splu_options=ddm.LOW_FILL) as P:
        t_factor = time.time() - t0
        print(f"factors: {t_factor:.1f} s wall over {P.workers} workers", flush=True)
        napply = [0]

        def Pinv(r):
            napply[0] += 1
            return P.apply(r)

        r0 = synth.rhs_for(w, 0)
        t0 = time.time()
        Pinv(r0)
        t_apply = time.time() - t0
        print(f"one application: {t_apply:.2f} s", flush=True)
        for k in rhs_ids:
            f = synth.rhs_for(w, k)
            nb = np.linalg.norm(f)

            def cb(it, est):
                if it % 25 == 0:
                    print(f"rhs {k} iter {it} est {est:.3e} ({time.time() - t1:.0f} s)", flush=True)
            t1 = time.time()
            x, info = gmres.gmres(A, Pinv, f, tol=w.tol, restart=3, maxit=5000, callback=cb)
            t_tol = time.time() - t1
            print(f"rhs {k}: {info['iters']} iterations to {info['relres_true']:.3e} in {t_tol:.0f} s",
                  flush=True)
            t1 = time.time()
            u, info2 = gmres.gmres(A, Pinv, f, tol=1e-10, restart=10, maxit=5000, x0=x, callback=cb)
            rel_ref = float(np.linalg.norm(f - A(u)) / nb)
            print(f"rhs {k}: reference after {info2['iters']} more iterations, relres {rel_ref:.3e}",
                  flush=True)
            rng = np.random.default_rng(12345 + k)
            iy = rng.integers(0, w.Ng, 4000)
            ix = rng.integers(0, w.Ng, 4000)
            out["rhs"][str(k)] = {
                "iters": int(info["iters"]),
                "restarts": int(info["restarts"]),
                "relres_true": float(info["relres_true"]),
                "ref_relres": rel_ref,
                "ref_extra_iters": int(info2["iters"]),
                "x_1e8_vs_ref_relL2": float(np.linalg.norm(x - u) / np.linalg.norm(u)),
                "u_norm": float(np.linalg.norm(u)),
                "samples": [[int(a), int(b), float(u[a, b].real), float(u[a, b].imag)]
                            for a, b in zip(iy, ix)],
                "oracle_seconds": {"factor_wall": t_factor, "one_apply": t_apply,
                                   "to_1e-8": t_tol, "reference": time.time() - t1},
                "workers": P.workers,
                "host_cpus": os.cpu_count(),
            }
            with open(PATH, "w") as fh:
                json.dump(out, fh)
            print(f"rhs {k} written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
