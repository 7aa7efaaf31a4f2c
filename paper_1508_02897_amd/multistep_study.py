"""The iterative multi-step DDM (Sec. 2, eq. ddms) as a solver against the
one-step preconditioner inside FGMRES (Sec. 3), on the same problems: steps
(preconditioner applications) and time to a relative residual tol.  The paper
finds the overlapping DDM more effective as a preconditioner than as a
solver.

    python -m paper_1508_02897_amd.multistep_study --workloads c1_128,c2_1024
"""
import argparse
import json
import os
import sys
import time


def run(name, max_steps, tol, device=0):
    import torch
    import synth
    from . import hddm as H
    from .solver import Solver, problem_from_workload
    w = synth.config(name)
    s = Solver(problem_from_workload(w, H.HDDM_MIXED_C64), synth.medium_for(w), device=device,
               restart=w.restart)
    s.factor()
    f = synth.rhs_for(w)
    out = {"workload": name, "tiles": f"{w.nb}x{w.nb}"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = s.ddm_solve(f, max_steps=max_steps, tol=tol, raise_on_noconv=False)
    torch.cuda.synchronize()
    out["ddm_steps"] = info["iters"]
    out["ddm_relres_true"] = info["relres_true"]
    out["ddm_converged"] = info["relres_est"] <= tol
    out["ddm_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = s.solve(f, tol=tol, restart=w.restart)
    torch.cuda.synchronize()
    out["fgmres_iters"] = info["iters"]
    out["fgmres_relres_true"] = info["relres_true"]
    out["fgmres_s"] = time.perf_counter() - t0
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="c1_128,c2_1024,c3_2048")
    ap.add_argument("--max-steps", type=int, default=3000)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    rows = []
    for name in args.workloads.split(","):
        r = run(name, args.max_steps, args.tol)
        rows.append(r)
        print(json.dumps(r), flush=True)
    print("| workload | tiles | multi-step DDM: steps | relres | time s | FGMRES(m): iterations "
          "| time s |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        steps = r["ddm_steps"] if r["ddm_converged"] else f">{r['ddm_steps']} (not converged)"
        print(f"| {r['workload']} | {r['tiles']} | {steps} | {r['ddm_relres_true']:.1e} | "
              f"{r['ddm_s']:.2f} | {r['fgmres_iters']} | {r['fgmres_s']:.2f} |", flush=True)


if __name__ == "__main__":
    main()
