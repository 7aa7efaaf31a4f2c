"""Overlap / PML-width study (Sec. 2 and the experiments with an extra overlap,
Tab. 4): the same problem solved with several overlap widths n_ol and local
PML widths P, reporting iterations against the bytes and time of the local
solves.  A wider overlap or layer makes the local problems closer to the
global one (fewer iterations) but larger (more factor bytes streamed per
application).  The paper reports fewer iterations with an extra overlap of 50
but a slower solve, and keeps no extra overlap.

Every run: complex64 factors, FP64 FGMRES(restart) to tol, one source, one
right-hand side (single form), the factor and the solve timed with the
library's own HIP events.  --smooth on|off|both solves with the smoothing
function of the Remark after eq. pc, without it (the default), or both.

--form block solves 16 sources together through the block form instead, with
the line factor (boxes up to 192 wide) or, --factor nd, the nested-dissection
factor (complex128 fronts, boxes whose fronts fit its kernels): the wide boxes
of an extra overlap then run in the block form too.

    python -m paper_1508_02897_amd.overlap_study --N 1280 --tile 160 \\
        --combos 0:16,8:16,50:16,0:30,8:30,50:30
"""
import argparse
import json
import os
import sys
import time


def run_block(N, tile, n_ol, P, medium, seed, ppw, restart, tol, fmt, nrhs=16, device=0):
    """The same problem solved for nrhs Gaussian sources together (block form)."""
    import numpy as np
    import torch
    import synth
    from . import hddm as H
    from .solver import Solver, problem_from_workload
    c_min = 0.8 if medium == "random" else 1.0
    w = synth.Workload(name=f"study_{N}_{tile}_{n_ol}_{P}", N=N, P=P, tile=tile, n_ol=n_ol,
                       ppw=ppw, c_min=c_min, medium=medium, medium_seed=seed, corr_len_h=20.0,
                       n_sources=1, source_seed=seed, restart=restart, tol=tol)
    ff = H.FORMAT_NESTED_DISSECTION if fmt == "nd" else H.FORMAT_AUTO
    s = Solver(problem_from_workload(w, H.HDDM_MIXED_C64, ff), synth.medium_for(w),
               device=device, restart=restart)
    nbx, nby, boxes = H.hddm_geometry(s.ctx)
    side = int(max((boxes[:, 1] - boxes[:, 0]).max(), (boxes[:, 3] - boxes[:, 2]).max()))
    centers = synth.gaussian_centers(N, nrhs, seed + 100)
    B = np.stack([synth.gaussian_rhs(N, P, centers[k:k + 1]) for k in range(nrhs)])
    s.ensure_block(nrhs, restart)
    H.hddm_profile(s.ctx, True)
    s.factor()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, infos = s.solve_block(B, tol=tol, restart=restart)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {k: H.hddm_profile_read(s.ctx, i) for i, k in enumerate(H.KERNEL_CLASSES)}
    H.hddm_profile(s.ctx, False)
    napp = max(prof["gather"][0], 1)
    iters = sorted(i["iters"] for i in infos)
    out = {
        "N": N, "tile": tile, "n_ol": n_ol, "P": P, "medium": medium, "form": "block",
        "factor": fmt, "nrhs": nrhs, "max_box_side": side, "factor_gb": s.factor_bytes / 1e9,
        "iters_median": iters[len(iters) // 2], "iters_max": iters[-1],
        "relres_true_max": max(i["relres_true"] for i in infos),
        "factor_ms": prof["factor"][1],
        "local_solves_ms_per_apply": prof["sweep"][1] / napp,
        "solve_s": wall, "solve_s_per_source": wall / nrhs,
    }
    s.close()
    return out


def run(N, tile, n_ol, P, medium, seed, ppw, restart, tol, smooth=False, device=0):
    import synth
    from . import hddm as H
    from .solver import Solver, problem_from_workload
    c_min = 0.8 if medium == "random" else 1.0
    w = synth.Workload(name=f"study_{N}_{tile}_{n_ol}_{P}", N=N, P=P, tile=tile, n_ol=n_ol,
                       ppw=ppw, c_min=c_min, medium=medium, medium_seed=seed, corr_len_h=20.0,
                       n_sources=1, source_seed=seed, restart=restart, tol=tol)
    s = Solver(problem_from_workload(w, H.HDDM_MIXED_C64), synth.medium_for(w), device=device,
               restart=restart)
    nbx, nby, boxes = H.hddm_geometry(s.ctx)
    side = int(max((boxes[:, 1] - boxes[:, 0]).max(), (boxes[:, 3] - boxes[:, 2]).max()))
    H.hddm_set_smoothing(s.ctx, smooth)
    H.hddm_profile(s.ctx, True)
    s.factor()
    f = synth.rhs_for(w)
    t0 = time.perf_counter()
    _, info = s.solve(f, tol=tol, restart=restart)
    import torch
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = {k: H.hddm_profile_read(s.ctx, i) for i, k in enumerate(H.KERNEL_CLASSES)}
    H.hddm_profile(s.ctx, False)
    nsw, sweep_ms = prof["sweep"]
    fb = s.factor_bytes
    out = {
        "N": N, "tile": tile, "n_ol": n_ol, "P": P, "medium": medium, "smooth": smooth,
        "boxes": nbx * nby,
        "max_box_side": side,
        # the library keeps complex64 factors symmetric-packed for boxes up to 256 wide
        "factor_format": "packed" if side <= 256 else "dense",
        "factor_gb": fb / 1e9,
        "iters": info["iters"], "relres_true": info["relres_true"],
        "factor_ms": prof["factor"][1],
        "sweep_ms_per_apply": sweep_ms / max(nsw, 1),
        "apply_ms_per_iter": (sweep_ms + prof["gather"][1]) / max(nsw, 1),
        "solve_s": wall,
    }
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=1280)
    ap.add_argument("--tile", type=int, default=160)
    ap.add_argument("--combos", default="0:16,8:16,50:16,0:30,8:30,50:30",
                    help="n_ol:P pairs")
    ap.add_argument("--medium", default="layered", choices=["layered", "random", "constant"])
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--ppw", type=float, default=10.0)
    ap.add_argument("--restart", type=int, default=50)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--smooth", default="off", choices=["off", "on", "both"])
    ap.add_argument("--form", default="single", choices=["single", "block"])
    ap.add_argument("--factor", default="line", choices=["line", "nd"],
                    help="block form: line factor or nested-dissection factor")
    args = ap.parse_args()
    smooths = {"off": [False], "on": [True], "both": [False, True]}[args.smooth]
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    rows = []
    if args.form == "block":
        for c in args.combos.split(","):
            n_ol, P = (int(x) for x in c.split(":"))
            r = run_block(args.N, args.tile, n_ol, P, args.medium, args.seed, args.ppw,
                          args.restart, args.tol, args.factor)
            rows.append(r)
            print(json.dumps(r), flush=True)
        print("| n_ol | P | factor | box side | factor GB | iterations (median / max) "
              "| local solves ms/apply | factor ms | solve s (16 sources) | s per source |")
        print("|---|---|---|---|---|---|---|---|---|---|")
        for r in rows:
            print(f"| {r['n_ol']} | {r['P']} | {r['factor']} | {r['max_box_side']} | "
                  f"{r['factor_gb']:.2f} | {r['iters_median']} / {r['iters_max']} | "
                  f"{r['local_solves_ms_per_apply']:.2f} | {r['factor_ms']:.0f} | "
                  f"{r['solve_s']:.2f} | {r['solve_s_per_source']:.3f} |", flush=True)
        return
    for c in args.combos.split(","):
        n_ol, P = (int(x) for x in c.split(":"))
        for sm in smooths:
            r = run(args.N, args.tile, n_ol, P, args.medium, args.seed, args.ppw, args.restart,
                    args.tol, sm)
            rows.append(r)
            print(json.dumps(r), flush=True)
    print("| n_ol | P | smoothing | box side | factor format | factor GB | iterations "
          "| sweep ms/apply | apply ms/iter | factor ms | solve s |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['n_ol']} | {r['P']} | {'on' if r['smooth'] else 'off'} | "
              f"{r['max_box_side']} | {r['factor_format']} | "
              f"{r['factor_gb']:.2f} | {r['iters']} | {r['sweep_ms_per_apply']:.2f} | "
              f"{r['apply_ms_per_iter']:.2f} | {r['factor_ms']:.0f} | {r['solve_s']:.2f} |",
              flush=True)


if __name__ == "__main__":
    main()
