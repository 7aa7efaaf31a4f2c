"""Writes <workload>_oracle.json for a large workload: the oracle's
DDM-preconditioned GMRES(50) iteration count to 1e-8 and the exact discrete
solution (sparse LU of the global PML system) at 2000 seeded sample nodes,
with its norm, and the residual estimate after every Arnoldi step.  Calls
only `oracle` and `synth`.
  c2_1024 (default): 1024^2 random medium, 8x8 boxes, 4 Gaussian sources;
                     a few minutes on a CPU.
  c3_2048:           2048^2 three-layer medium, 16x16 boxes, 1 Gaussian
                     source; about an hour and ~25 GB of memory.
Run from the repository root:  python tests/golden/make_golden_large.py [c3_2048]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import synth  # noqa: E402
from oracle import Problem, direct, gmres  # noqa: E402


DESCRIPTION = {
    "c2_1024": "1024^2 interior, P=16, 8x8 tiles of 128, n_ol=8, random medium corr 20h seed 2, "
               "10 ppw at c=0.8, 4 Gaussian sources seed 2, GMRES(50) tol 1e-8",
    "c3_2048": "2048^2 interior, P=16, 16x16 tiles of 128, n_ol=8, three-layer medium seed 3, "
               "12 ppw at c=1.0, 1 Gaussian source seed 3, GMRES(50) tol 1e-8",
}


def main(name="c2_1024"):
    w = synth.config(name)
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    t0 = time.time()
    u = direct.sparse_solve(prob, f)
    t_direct = time.time() - t0
    t0 = time.time()
    x, info = gmres.solve(prob, f, tol=w.tol, restart=w.restart)
    t_gmres = time.time() - t0
    rng = np.random.default_rng(12345)
    iy = rng.integers(0, w.Ng, 2000)
    ix = rng.integers(0, w.Ng, 2000)
    out = {
        "workload": DESCRIPTION[name],
        "iters": int(info["iters"]),
        "relres_true": float(info["relres_true"]),
        # the residual estimate |gamma_{j+1}| / |b| after every Arnoldi step
        "history": [float(v) for v in info["history"]],
        "gmres_vs_direct_relL2": float(np.linalg.norm(x - u) / np.linalg.norm(u)),
        "u_norm": float(np.linalg.norm(u)),
        "samples": [[int(a), int(b), float(u[a, b].real), float(u[a, b].imag)] for a, b in zip(iy, ix)],
        "oracle_seconds": {"direct": t_direct, "gmres": t_gmres},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print({k: out[k] for k in ("iters", "relres_true", "gmres_vs_direct_relL2", "u_norm", "oracle_seconds")})


if __name__ == "__main__":
    main(*sys.argv[1:2])
