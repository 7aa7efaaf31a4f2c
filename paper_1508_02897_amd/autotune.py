"""Autotuner: times the library's kernel variants on the caller's own problem
through the C ABI (hddm_tune + hddm_profile) and keeps the fastest.

Candidates: the complex64 factor on MFMA (symmetric elimination, full
elimination with the working matrix in registers or in memory) or on vector
FMA; the complex64 sweep
as the wave-structured kernel (one workgroup per CU, block prefetch) or the
one-row-per-thread kernel at several workgroup sizes; the block sweep (16
right-hand sides per step) with three or four real MFMAs per complex product.
The sweep variants share one factorisation (they read the same layout), so
tuning costs four factors and a few preconditioner applications.

The choices can be kept in a JSON cache (`tune_cached`), keyed by the device,
the precision, the local-solver format, the box count and the largest box:
the kernel times depend on those shapes, not on the medium, so a later setup
of the same shape applies the stored choice without timing anything.

    python -m paper_1508_02897_amd.autotune --workload c4_4096 --precision mixed [--block]
        [--cache PATH]
"""
import argparse
import json
import os
import sys
import tempfile

from . import hddm as H

THREADS = (0, 448, 704, 1024)


def _apply_ms(solver, r, z, applies):
    solver.apply_precond(r, out=z)  # warm
    H.hddm_profile(solver.ctx, True)
    for _ in range(applies):
        solver.apply_precond(r, out=z)
    n, ms = H.hddm_profile_read(solver.ctx, H.HDDM_K_SWEEP)
    H.hddm_profile(solver.ctx, False)
    return ms / max(n, 1)


def tune(solver, applies=2, threads=THREADS, verbose=False):
    """Select the fastest factor and sweep variants for `solver` (which must be
    bound); leaves the problem factored with the chosen factor.  Returns a dict
    of the measured times and the choice."""
    import torch
    ctx = solver.ctx
    mixed = solver.prob.precision == H.HDDM_MIXED_C64
    pr = solver.prob
    single = pr.nx == pr.tile and pr.ny == pr.tile  # one box: the whole grid
    max_side = max(solver.ngx, solver.ngy) if single else pr.tile + 2 * (pr.n_ol + pr.npml)
    out = {"factor_ms": {}, "sweep_ms": {}}
    best_f = H.FACTOR_AUTO
    if mixed:
        cands = ((H.FACTOR_AUTO, "mfma"), (H.FACTOR_MFMA_REGS, "mfma_full_elimination"),
                 (H.FACTOR_VECTOR, "vector"), (H.FACTOR_MFMA_MEM, "mfma_memory_working_matrix"))
        for fv, name in cands:
            H.hddm_tune(ctx, H.SWEEP_AUTO, 0, fv)
            H.hddm_profile(ctx, True)
            solver.factor()
            _, ms = H.hddm_profile_read(ctx, H.HDDM_K_FACTOR)
            H.hddm_profile(ctx, False)
            out["factor_ms"][name] = ms
            if verbose:
                print(f"factor {name:8s} {ms:9.2f} ms", flush=True)
        best_f = min(((fv, out["factor_ms"][name]) for fv, name in cands),
                     key=lambda t: t[1])[0]
    H.hddm_tune(ctx, H.SWEEP_AUTO, 0, best_f)
    solver.factor()
    g = torch.Generator(device=solver.device).manual_seed(0)
    r = torch.randn((solver.ngy, solver.ngx), dtype=torch.complex128, device=solver.device,
                    generator=g)
    z = solver.empty()
    packed = mixed and solver.prob.factor_format == 0 and max_side <= 256
    if packed:  # symmetric-packed format: one or two workgroups per CU
        cands = [(H.SWEEP_AUTO, 0), (H.SWEEP_WAVE, 0)]
    else:
        cands = [(H.SWEEP_ROW, t) for t in threads]
        if mixed and max_side <= 192:
            cands.insert(0, (H.SWEEP_WAVE, 0))
    best = None
    for sv, th in cands:
        H.hddm_tune(ctx, sv, th, best_f)
        ms = _apply_ms(solver, r, z, applies)
        if packed:
            key = "packed_two_per_cu" if sv == H.SWEEP_WAVE else "packed_one_per_cu"
        else:
            key = "wave" if sv == H.SWEEP_WAVE else f"row_threads_{th or 'auto'}"
        out["sweep_ms"][key] = ms
        if verbose:
            print(f"sweep  {key:18s} {ms:9.3f} ms", flush=True)
        if best is None or ms < best[2]:
            best = (sv, th, ms)
    H.hddm_tune(ctx, best[0], best[1], best_f)
    out["choice"] = {"sweep_variant": best[0], "sweep_threads": best[1], "factor_variant": best_f}
    return out


def tune_block(solver, applies=2, verbose=False):
    """Select the fastest complex64 factor (symmetric or full elimination in
    registers, boxes up to 192 wide) and block-sweep kernel (three or four
    real MFMAs per complex product, transposed operand from LDS or memory)
    for `solver`, leaving it factored with the chosen factor; returns the
    times and choice."""
    import torch
    ctx = solver.ctx
    out = {"factor_ms": {}, "block_sweep_ms": {}}
    width = max(int(b[1] - b[0]) for b in H.hddm_geometry(ctx)[2])
    fcands = ((H.FACTOR_AUTO, "mfma"), (H.FACTOR_MFMA_REGS, "mfma_full_elimination"))
    best_f = (H.FACTOR_AUTO, None)
    for fv, name in (fcands if width <= 192 else fcands[:1]):
        H.hddm_tune(ctx, H.SWEEP_AUTO, 0, fv)
        H.hddm_profile(ctx, True)
        solver.factor()
        _, ms = H.hddm_profile_read(ctx, H.HDDM_K_FACTOR)
        H.hddm_profile(ctx, False)
        out["factor_ms"][name] = ms
        if verbose:
            print(f"factor {name:26s} {ms:9.2f} ms", flush=True)
        if best_f[1] is None or ms < best_f[1]:
            best_f = (fv, ms)
    H.hddm_tune(ctx, H.SWEEP_AUTO, 0, best_f[0])
    solver.factor()
    g = torch.Generator(device=solver.device).manual_seed(0)
    R = torch.randn((H.HDDM_BLOCK_MAX, solver.ngy, solver.ngx), dtype=torch.complex128,
                    device=solver.device, generator=g)
    Z = torch.empty_like(R)
    best = None
    for variant, key in ((H.BLOCK_3M, "three_mfma_lds_transpose"), (H.BLOCK_4M, "four_mfma"),
                         (H.BLOCK_3M_MEMT, "three_mfma")):
        H.hddm_tune_block(ctx, variant)
        solver.apply_precond_block(R, out=Z)  # warm
        H.hddm_profile(ctx, True)
        for _ in range(applies):
            solver.apply_precond_block(R, out=Z)
        n, ms = H.hddm_profile_read(ctx, H.HDDM_K_SWEEP)
        H.hddm_profile(ctx, False)
        ms /= max(n, 1)
        out["block_sweep_ms"][key] = ms
        if verbose:
            print(f"block sweep {key:26s} {ms:9.3f} ms", flush=True)
        if best is None or ms < best[1]:
            best = (variant, ms)
    H.hddm_tune_block(ctx, best[0])
    out["choice"] = {"block_variant": best[0], "factor_variant": best_f[0]}
    return out


def cache_key(device_name, precision, factor_format, nbx, nby, max_mx, max_my, block):
    """Key of a tuning result: what the kernel times depend on."""
    prec = "c64" if precision == H.HDDM_MIXED_C64 else "c128"
    form = "block" if block else "single"
    return (f"{device_name}|{prec}|format{factor_format}|boxes{nbx}x{nby}|"
            f"box{max_mx}x{max_my}|{form}")


def load_cache(path):
    """The cache's entries ({} if the file does not exist)."""
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_cache(path, entries):
    """Write the entries atomically (a partly written cache is never read)."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def solver_key(solver, block):
    import torch
    nbx, nby, boxes = H.hddm_geometry(solver.ctx)
    max_mx = int((boxes[:, 1] - boxes[:, 0]).max())
    max_my = int((boxes[:, 3] - boxes[:, 2]).max())
    name = torch.cuda.get_device_properties(solver.device).name
    return cache_key(name, solver.prob.precision, solver.prob.factor_format, nbx, nby, max_mx,
                     max_my, block)


def apply_choice(solver, choice, block):
    """Select the stored kernels and refactor with the stored factor variant."""
    fv = choice.get("factor_variant", H.FACTOR_AUTO)
    H.hddm_tune(solver.ctx, choice.get("sweep_variant", H.SWEEP_AUTO),
                choice.get("sweep_threads", 0), fv)
    if block:
        H.hddm_tune_block(solver.ctx, choice["block_variant"])
    solver.factor()


def tune_cached(solver, path, block=False, **kw):
    """tune / tune_block through the JSON cache at `path`: a stored choice for
    this shape is applied (and the problem refactored with its factor
    variant); otherwise the tuner runs and its result is stored.  Returns the
    result with "cached": True or False."""
    key = solver_key(solver, block)
    entries = load_cache(path)
    if key in entries:
        res = dict(entries[key])
        apply_choice(solver, res["choice"], block)
        res["cached"] = True
        return res
    if block:
        solver.factor()
        res = tune_block(solver, **kw)
    else:
        res = tune(solver, **kw)
    entries = load_cache(path)  # another process may have written meanwhile
    entries[key] = res
    save_cache(path, entries)
    return dict(res, cached=False)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c4_4096")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "plain"])
    ap.add_argument("--applies", type=int, default=2)
    ap.add_argument("--block", action="store_true", help="tune the block sweep instead")
    ap.add_argument("--cache", default=None,
                    help="JSON cache of tuning results: apply a stored choice for this shape, "
                         "or tune and store it")
    args = ap.parse_args()
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth
    from .solver import Solver, problem_from_workload
    w = synth.config(args.workload)
    prec = H.HDDM_MIXED_C64 if args.precision == "mixed" else H.HDDM_PLAIN_C128
    s = Solver(problem_from_workload(w, prec), synth.medium_for(w), restart=1)
    print(f"# {w.name} precision={args.precision}", flush=True)
    if args.cache:
        res = tune_cached(s, args.cache, block=args.block, applies=args.applies, verbose=True)
    elif args.block:
        s.factor()
        res = tune_block(s, applies=args.applies, verbose=True)
    else:
        res = tune(s, applies=args.applies, verbose=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
