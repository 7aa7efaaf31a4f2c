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

    python -m paper_1508_02897_amd.overlap_study --N 1280 --tile 160 \\
        --combos 0:16,8:16,50:16,0:30,8:30,50:30
"""
import argparse
import json
import os
import sys
import time


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
    args = ap.parse_args()
    smooths = {"off": [False], "on": [True], "both": [False, True]}[args.smooth]
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    rows = []
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
