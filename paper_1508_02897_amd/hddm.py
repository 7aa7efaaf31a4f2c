"""ctypes binding of the C ABI in include/hddm.h: the same entry points, with
argument marshalling only.  Device buffers are torch tensors (memory and
streams); all arithmetic runs in libhddm.so.  Importing works without a GPU;
calling anything that needs the library raises if libhddm.so is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhddm.so")

HDDM_OK, HDDM_EINVAL, HDDM_ENOMEM, HDDM_ESTATE, HDDM_ENOCONV, HDDM_EBREAKDOWN, HDDM_EDEVICE = range(7)
HDDM_PLAIN_C128, HDDM_MIXED_C64 = 0, 1
# Problem.factor_format: packed (complex64) or dense line factors, or the
# nested-dissection multifrontal factor (complex128 fronts, complex64 vectors)
FORMAT_AUTO, FORMAT_DENSE, FORMAT_NESTED_DISSECTION = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "ESTATE", 4: "ENOCONV", 5: "EBREAKDOWN",
                6: "EDEVICE"}

# every function declared in include/hddm.h
EXPORTS = ("hddm_setup", "hddm_query_bytes", "hddm_bind", "hddm_factor", "hddm_apply_precond",
           "hddm_matvec", "hddm_solve", "hddm_destroy", "hddm_last_error", "hddm_geometry",
           "hddm_stretch_tables", "hddm_tune", "hddm_profile", "hddm_profile_read",
           "hddm_share_factor", "hddm_query_block_bytes", "hddm_apply_precond_block",
           "hddm_solve_block", "hddm_tune_block", "hddm_use_graphs", "hddm_set_smoothing",
           "hddm_ddm_query_bytes", "hddm_ddm_solve", "hddm_apply_precond_noalloc", "hddm_factor_pivots",
           "hddm_apply_precond_batch", "hddm_session_create", "hddm_session_add",
           "hddm_session_step", "hddm_session_result", "hddm_session_destroy",
           "hddm_solve_history")
HDDM_BATCH_MAX = 8
HDDM_K_SWEEP, HDDM_K_GATHER, HDDM_K_MATVEC, HDDM_K_KRYLOV, HDDM_K_FACTOR, HDDM_K_RESTRICT = range(6)
KERNEL_CLASSES = ("sweep", "gather", "matvec", "krylov", "factor", "restrict")
HDDM_BLOCK_MAX = 16


class HddmError(RuntimeError):
    def __init__(self, status, msg, info=None):
        super().__init__(f"hddm {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.info = info


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("npml", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("n_ol", ctypes.c_int32), ("pml_power", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("factor_format", ctypes.c_int32),
                ("h", ctypes.c_double), ("omega", ctypes.c_double), ("k_ref", ctypes.c_double),
                ("sigma0_over_kref", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("ortho", ctypes.c_int32), ("reserved", ctypes.c_int32)]

ORTHO_CGS2, ORTHO_CGS2_GRAM = 0, 1


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "restarts": self.restarts, "relres_est": self.relres_est,
                "relres_true": self.relres_true, "status": STATUS_NAMES.get(self.status, self.status)}


_lib = None


def lib():
    """The loaded libhddm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1508_02897_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        L.hddm_setup.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_double), i32,
                                 ctypes.POINTER(vp)]
        L.hddm_query_bytes.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz),
                                       ctypes.POINTER(sz)]
        L.hddm_bind.argtypes = [vp, vp, sz, vp, sz, vp]
        L.hddm_factor.argtypes = [vp, vp]
        L.hddm_apply_precond.argtypes = [vp, vp, vp, vp]
        L.hddm_apply_precond_noalloc.argtypes = [vp, vp, vp, vp]
        L.hddm_matvec.argtypes = [vp, vp, vp, vp]
        L.hddm_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo),
                                 vp, sz, vp]
        L.hddm_destroy.argtypes = [vp]
        L.hddm_last_error.argtypes = []
        L.hddm_last_error.restype = ctypes.c_char_p
        L.hddm_geometry.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]
        L.hddm_stretch_tables.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.hddm_tune.argtypes = [vp, i32, i32, i32]
        L.hddm_share_factor.argtypes = [vp, vp]
        L.hddm_factor_pivots.argtypes = [vp, ctypes.POINTER(ctypes.c_float), vp]
        P, i64 = ctypes.POINTER, ctypes.c_int64
        L.hddm_apply_precond_batch.argtypes = [P(vp), i32, P(vp), P(i64), P(vp), P(i64), P(i32),
                                               P(vp), P(sz), vp]
        L.hddm_session_create.argtypes = [P(vp)]
        L.hddm_session_add.argtypes = [vp, vp, vp, i64, vp, i64, i32, P(SolveOpts), vp, sz, vp,
                                       sz, P(i32)]
        L.hddm_session_step.argtypes = [vp, vp, P(i32), P(i32)]
        L.hddm_session_result.argtypes = [vp, i32, P(SolveInfo)]
        L.hddm_session_destroy.argtypes = [vp]
        i64 = ctypes.c_int64
        L.hddm_query_block_bytes.argtypes = [vp, i32, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.hddm_apply_precond_block.argtypes = [vp, vp, i64, vp, i64, i32, vp, sz, vp]
        L.hddm_solve_block.argtypes = [vp, vp, i64, vp, i64, i32, ctypes.POINTER(SolveOpts),
                                       ctypes.POINTER(SolveInfo), vp, sz, vp, sz, vp]
        L.hddm_tune_block.argtypes = [vp, i32]
        L.hddm_use_graphs.argtypes = [vp, i32]
        L.hddm_set_smoothing.argtypes = [vp, i32]
        L.hddm_ddm_query_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.hddm_ddm_solve.argtypes = [vp, vp, vp, i32, ctypes.c_double, ctypes.POINTER(SolveInfo),
                                     vp, sz, vp]
        L.hddm_profile.argtypes = [vp, i32]
        L.hddm_solve_history.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), i32,
                                         ctypes.POINTER(i32)]
        L.hddm_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
        for name in EXPORTS:
            if name != "hddm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status, info=None):
    if status != HDDM_OK:
        raise HddmError(status, lib().hddm_last_error().decode(), info)


def hddm_last_error():
    return lib().hddm_last_error().decode()


def hddm_setup(prob, velocity, device=0):
    vel = np.ascontiguousarray(velocity, dtype=np.float64)
    ctx = ctypes.c_void_p()
    _check(lib().hddm_setup(ctypes.byref(prob), vel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            int(device), ctypes.byref(ctx)))
    return ctx


def hddm_query_bytes(ctx, restart):
    f, w, k = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().hddm_query_bytes(ctx, int(restart), ctypes.byref(f), ctypes.byref(w), ctypes.byref(k)))
    return f.value, w.value, k.value


def hddm_bind(ctx, factor_ptr, factor_bytes, work_ptr, work_bytes, stream=0):
    _check(lib().hddm_bind(ctx, factor_ptr, factor_bytes, work_ptr, work_bytes, stream))


def hddm_factor(ctx, stream=0):
    _check(lib().hddm_factor(ctx, stream))


def hddm_apply_precond(ctx, r_ptr, z_ptr, stream=0):
    _check(lib().hddm_apply_precond(ctx, r_ptr, z_ptr, stream))


def hddm_apply_precond_noalloc(ctx, r_ptr, z_ptr, stream=0):
    _check(lib().hddm_apply_precond_noalloc(ctx, r_ptr, z_ptr, stream))


def hddm_matvec(ctx, x_ptr, y_ptr, stream=0):
    _check(lib().hddm_matvec(ctx, x_ptr, y_ptr, stream))


def hddm_solve(ctx, rhs_ptr, x_ptr, opts, krylov_ptr, krylov_bytes, stream=0, raise_on_noconv=True):
    info = SolveInfo()
    st = lib().hddm_solve(ctx, rhs_ptr, x_ptr, ctypes.byref(opts), ctypes.byref(info), krylov_ptr,
                          krylov_bytes, stream)
    if st == HDDM_ENOCONV and not raise_on_noconv:
        return info
    _check(st, info)
    return info


def hddm_ddm_query_bytes(ctx):
    w = ctypes.c_size_t()
    _check(lib().hddm_ddm_query_bytes(ctx, ctypes.byref(w)))
    return w.value


def hddm_ddm_solve(ctx, rhs_ptr, x_ptr, max_steps, tol, work_ptr, work_bytes, stream=0,
                   raise_on_noconv=True):
    info = SolveInfo()
    st = lib().hddm_ddm_solve(ctx, rhs_ptr, x_ptr, int(max_steps), float(tol), ctypes.byref(info),
                              work_ptr, work_bytes, stream)
    if st == HDDM_ENOCONV and not raise_on_noconv:
        return info
    _check(st, info)
    return info


def hddm_query_block_bytes(ctx, nrhs, restart):
    w, k = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().hddm_query_block_bytes(ctx, int(nrhs), int(restart), ctypes.byref(w),
                                        ctypes.byref(k)))
    return w.value, k.value


def hddm_apply_precond_block(ctx, r_ptr, ldr, z_ptr, ldz, nrhs, work_ptr, work_bytes, stream=0):
    _check(lib().hddm_apply_precond_block(ctx, r_ptr, int(ldr), z_ptr, int(ldz), int(nrhs),
                                          work_ptr, work_bytes, stream))


def hddm_solve_block(ctx, rhs_ptr, ldb, x_ptr, ldx, nrhs, opts, work_ptr, work_bytes, krylov_ptr,
                     krylov_bytes, stream=0, raise_on_noconv=True):
    infos = (SolveInfo * int(nrhs))()
    st = lib().hddm_solve_block(ctx, rhs_ptr, int(ldb), x_ptr, int(ldx), int(nrhs),
                                ctypes.byref(opts), infos, work_ptr, work_bytes, krylov_ptr,
                                krylov_bytes, stream)
    if st == HDDM_ENOCONV and not raise_on_noconv:
        return list(infos)
    _check(st, list(infos))
    return list(infos)


def hddm_solve_history(ctx, rhs=0):
    """Residual estimates after every Arnoldi step of the context's last
    completed solve (right-hand side `rhs`), as a float64 array."""
    n = ctypes.c_int32()
    _check(lib().hddm_solve_history(ctx, int(rhs), None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=np.float64)
    if n.value:
        _check(lib().hddm_solve_history(ctx, int(rhs),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        n.value, ctypes.byref(n)))
    return out


def hddm_destroy(ctx):
    _check(lib().hddm_destroy(ctx))


def hddm_geometry(ctx):
    nbx, nby = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hddm_geometry(ctx, ctypes.byref(nbx), ctypes.byref(nby), None))
    boxes = np.zeros((nbx.value * nby.value, 8), dtype=np.int32)
    _check(lib().hddm_geometry(ctx, ctypes.byref(nbx), ctypes.byref(nby),
                               boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return nbx.value, nby.value, boxes


def hddm_stretch_tables(ctx, ngx, ngy):
    out = np.zeros(2 * (2 * ngx + 1 + 2 * ngy + 1), dtype=np.float64)
    _check(lib().hddm_stretch_tables(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    c = out.view(np.complex128)
    ax = c[:ngx]; hx = c[ngx:2 * ngx + 1]
    ay = c[2 * ngx + 1:2 * ngx + 1 + ngy]; hy = c[2 * ngx + 1 + ngy:]
    return ax, hx, ay, hy


def hddm_profile(ctx, enable):
    _check(lib().hddm_profile(ctx, 1 if enable else 0))


def hddm_profile_read(ctx, kernel):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().hddm_profile_read(ctx, int(kernel), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


SWEEP_AUTO, SWEEP_WAVE, SWEEP_ROW = 0, 1, 2
FACTOR_AUTO, FACTOR_VECTOR, FACTOR_MFMA_MEM, FACTOR_MFMA_REGS, FACTOR_MFMA_SYM = 0, 1, 2, 3, 4


def hddm_tune(ctx, sweep_variant=0, sweep_threads=0, factor_variant=0):
    _check(lib().hddm_tune(ctx, int(sweep_variant), int(sweep_threads), int(factor_variant)))


BLOCK_AUTO, BLOCK_3M, BLOCK_4M, BLOCK_3M_MEMT = 0, 1, 2, 3


def hddm_set_smoothing(ctx, enable=True):
    _check(lib().hddm_set_smoothing(ctx, 1 if enable else 0))


def hddm_use_graphs(ctx, enable=True):
    _check(lib().hddm_use_graphs(ctx, 1 if enable else 0))


def hddm_tune_block(ctx, variant=BLOCK_AUTO):
    _check(lib().hddm_tune_block(ctx, int(variant)))


def hddm_factor_pivots(ctx, nboxes, stream=0):
    """(nboxes, 2) array: smallest and largest pivot magnitude per box."""
    out = np.zeros((int(nboxes), 2), dtype=np.float32)
    _check(lib().hddm_factor_pivots(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream))
    return out


def _arr(ctype, vals):
    return (ctype * len(vals))(*vals)


def hddm_apply_precond_batch(ctxs, r_ptrs, ldr, z_ptrs, ldz, nrhs, work_ptrs, work_bytes,
                             stream=0):
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    _check(lib().hddm_apply_precond_batch(
        _arr(vp, [c.value if isinstance(c, vp) else c for c in ctxs]), len(ctxs),
        _arr(vp, r_ptrs), _arr(i64, ldr), _arr(vp, z_ptrs), _arr(i64, ldz), _arr(i32, nrhs),
        _arr(vp, work_ptrs), _arr(sz, work_bytes), stream))


def hddm_session_create():
    s = ctypes.c_void_p()
    _check(lib().hddm_session_create(ctypes.byref(s)))
    return s


def hddm_session_add(sess, ctx, rhs_ptr, ldb, x_ptr, ldx, nrhs, opts, work_ptr, work_bytes,
                     krylov_ptr, krylov_bytes):
    pid = ctypes.c_int32()
    _check(lib().hddm_session_add(sess, ctx, rhs_ptr, int(ldb), x_ptr, int(ldx), int(nrhs),
                                  ctypes.byref(opts), work_ptr, work_bytes, krylov_ptr,
                                  krylov_bytes, ctypes.byref(pid)))
    return pid.value


def hddm_session_step(sess, stream=0):
    """One round of every problem; returns the ids of those that finished."""
    done = (ctypes.c_int32 * HDDM_BATCH_MAX)()
    nd = ctypes.c_int32()
    _check(lib().hddm_session_step(sess, stream, done, ctypes.byref(nd)))
    return list(done[:nd.value])


def hddm_session_result(sess, pid, nrhs, raise_on_noconv=True):
    infos = (SolveInfo * int(nrhs))()
    st = lib().hddm_session_result(sess, int(pid), infos)
    if st == HDDM_ENOCONV and not raise_on_noconv:
        return list(infos)
    _check(st, list(infos))
    return list(infos)


def hddm_session_destroy(sess):
    _check(lib().hddm_session_destroy(sess))


def hddm_share_factor(dst, src):
    _check(lib().hddm_share_factor(dst, src))
