"""Host logic of the benchmark (no GPU): the algorithmic work that the
roofline fields divide by, counted here independently step by step on small
boxes, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _sweep_by_steps(boxes, nrhs, flops_per_cmac):
    """Walk the two sweeps of every box: each step multiplies one stored
    block (mx x mx, packed 16x16 upper tiles) by an mx x nrhs panel, reading
    the off-diagonal tiles whole and the diagonal tiles' upper triangles."""
    flops = byts = 0.0
    for bx0, bx1, by0, by1, tx0, tx1, ty0, ty1 in boxes:
        mx, my = bx1 - bx0, by1 - by0
        nt = -(-mx // 16)
        packed = sum(256 if I < J else 16 * 17 // 2 for J in range(nt) for I in range(J + 1))
        j0 = ty0 - by0
        fwd = list(range(j0, my))            # forward from the first tile row
        bwd = list(range(my - 2, -1, -1))    # backward over the other rows
        for j in fwd + bwd:
            flops += flops_per_cmac * mx * mx * nrhs
            byts += 8 * packed
        # complex64 workspace: the sources of the tile rows read, the forward
        # results written, read back by the backward sweep for rows j0 .. my-2
        # (row my-1 is final after the forward sweep), the solution rows written
        byts += 8 * nrhs * mx * (ty1 - ty0)
        byts += 8 * nrhs * mx * len(fwd)
        byts += 8 * nrhs * mx * (len(fwd) - 1)
        byts += 8 * nrhs * mx * len(bwd)
    return flops, byts


def test_block_sweep_work_matches_step_count():
    boxes = [(0, 52, 0, 52, 8, 40, 8, 40), (40, 96, 28, 84, 44, 76, 40, 72),
             (0, 40, 0, 33, 3, 37, 5, 30)]
    for fpc in (6, 8):
        f, b = bench.block_sweep_work(boxes, 16, flops_per_cmac=fpc)
        f2, b2 = _sweep_by_steps(boxes, 16, fpc)
        assert f == f2
        assert b == b2


def test_factor_flops_hand_count():
    # one 176 x 168 box and one 104 x 104 box: 8 mx^3 flops per x-line for
    # the full elimination, half of it for the symmetric one
    boxes = [(0, 176, 0, 168), (10, 114, 20, 124)]
    full = 8 * 176 ** 3 * 168 + 8 * 104 ** 3 * 104
    assert bench.factor_flops(boxes, symmetric=False) == full
    assert bench.factor_flops(boxes) == full / 2


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout
