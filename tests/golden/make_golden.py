"""Writes c1_oracle.json: the oracle's GMRES iteration count and direct-solve
samples for the 128^2 constant-medium workload.  Calls only `oracle` and
`synth`.  Run from the repository root:  python tests/golden/make_golden.py"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import synth  # noqa: E402
from oracle import Problem, direct, gmres  # noqa: E402


def main():
    w = synth.config("c1_128")
    prob = Problem.from_workload(w)
    f = synth.rhs_for(w)
    x, info = gmres.solve(prob, f, tol=w.tol, restart=w.restart)
    u = direct.banded_solve(prob, f)
    pts = [(16, 16), (80, 80), (40, 120), (150, 7), (100, 63)]
    out = {
        "workload": "128^2 interior, P=16, 2x2 tiles of 64, n_ol=8, c=1, 10 ppw, GMRES(50) tol 1e-8",
        "iters": int(info["iters"]),
        "relres_true": float(info["relres_true"]),
        "samples": [[iy, ix, float(u[iy, ix].real), float(u[iy, ix].imag)] for iy, ix in pts],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
