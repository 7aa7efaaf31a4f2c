"""Local direct solver study (Sec. 3: the local problems are factorised once
by a direct solver and reused): the line-by-line block factor (G_j = S_j^-1
of the x-lines, symmetric-packed complex64) against the low-fill
nested-dissection multifrontal factor (complex128 fronts), on the same
workload in the block form (16 right-hand sides per application): factor
bytes and time, time of one application's local solves, and the solve.

Every run: precision HDDM_MIXED_C64, FP64 FGMRES(restart) with the Gram-matrix
CGS2 to the workload's tolerance, the workload's first nrhs sources; kernel
times from the library's own HIP events.

    python -m paper_1508_02897_amd.local_solver_study --workload c4_4096
"""
import argparse
import json
import os
import sys
import time

FORMATS = {"line": 0, "nested_dissection": 2}


def run(name, fmt, nrhs=16, restart=3, applies=5, solve=True, device=0):
    import numpy as np
    import torch
    import synth
    from . import hddm as H
    from .solver import Solver, problem_from_workload
    w = synth.config(name)
    s = Solver(problem_from_workload(w, H.HDDM_MIXED_C64, FORMATS[fmt]), synth.medium_for(w),
               device=device, restart=restart)
    dev = torch.device("cuda", device)
    B = torch.from_numpy(np.stack([synth.rhs_for(w, k % w.n_rhs) for k in range(nrhs)])).to(dev)
    s.ensure_block(nrhs, restart)
    out = {"workload": name, "local_solver": fmt, "nrhs": nrhs, "restart": restart,
           "factor_gb": s.factor_bytes / 1e9}

    def prof():
        return {k: H.hddm_profile_read(s.ctx, i) for i, k in enumerate(H.KERNEL_CLASSES)}

    H.hddm_profile(s.ctx, True)
    s.factor()
    torch.cuda.synchronize()
    out["factor_ms"] = prof()["factor"][1]
    Z = torch.empty_like(B)
    s.apply_precond_block(B, out=Z)  # first launch builds the graph
    H.hddm_profile(s.ctx, False)
    H.hddm_profile(s.ctx, True)
    for _ in range(applies):
        s.apply_precond_block(B, out=Z)
    torch.cuda.synchronize()
    p = prof()
    napp = max(p["gather"][0], 1)
    out["local_solves_ms_per_apply"] = p["sweep"][1] / napp
    out["sweep_launches_per_apply"] = p["sweep"][0] / napp
    out["gather_ms_per_apply"] = p["gather"][1] / napp
    H.hddm_profile(s.ctx, False)
    if not solve:
        s.close()
        return out
    X = torch.empty_like(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos = s.solve_block(B, tol=w.tol, restart=restart, out=X, raise_on_noconv=False)
    torch.cuda.synchronize()
    out["solve_s"] = time.perf_counter() - t0
    out["iters"] = [i["iters"] for i in infos]
    out["relres_true_max"] = max(i["relres_true"] for i in infos)
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c4_4096")
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--restart", type=int, default=3)
    ap.add_argument("--formats", default="line,nested_dissection")
    ap.add_argument("--no-solve", action="store_true",
                    help="factor and time the applications only (for profiler runs)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    rows = []
    for fmt in args.formats.split(","):
        r = run(args.workload, fmt, args.nrhs, args.restart, solve=not args.no_solve)
        rows.append(r)
        print(json.dumps(r), flush=True)
    if args.no_solve:
        return
    print("| local solver | factor GB | factor ms | local solves ms/apply (launches) "
          "| gather ms/apply | iterations (min-max) | max relres | solve s |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['local_solver']} | {r['factor_gb']:.1f} | {r['factor_ms']:.0f} | "
              f"{r['local_solves_ms_per_apply']:.2f} ({r['sweep_launches_per_apply']:.0f}) | "
              f"{r['gather_ms_per_apply']:.2f} | {min(r['iters'])}-{max(r['iters'])} | "
              f"{r['relres_true_max']:.1e} | {r['solve_s']:.2f} |", flush=True)


if __name__ == "__main__":
    main()
