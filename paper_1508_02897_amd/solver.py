"""Convenience wrapper over the C ABI: owns the torch device buffers of one
medium (factor, work, Krylov) and forwards every call to libhddm.so."""
import numpy as np
import torch

from . import hddm as H


def make_problem(nx, ny, npml, tile, n_ol, h, omega, k_ref, sigma0_over_kref=20.0, pml_power=2,
                 precision=H.HDDM_PLAIN_C128, factor_format=0):
    return H.Problem(nx=nx, ny=ny, npml=npml, tile=tile, n_ol=n_ol, pml_power=pml_power,
                     precision=precision, factor_format=factor_format, h=h, omega=omega,
                     k_ref=k_ref, sigma0_over_kref=sigma0_over_kref)


def problem_from_workload(w, precision=H.HDDM_PLAIN_C128, factor_format=0):
    return make_problem(w.N, w.N, w.P, w.tile, w.n_ol, w.h, w.omega, w.k_ref,
                        w.sigma0_over_kref, w.pml_power, precision, factor_format)


def _stream(device):
    return torch.cuda.current_stream(device).cuda_stream


def _buf(nbytes, device):
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Solver:
    """One medium on one GPU: setup -> bind -> factor, then apply/matvec/solve."""

    def __init__(self, prob, velocity, device=0, restart=50, share_from=None):
        """share_from: another Solver of the same problem whose factor buffer
        (and, once factored, factorisation) this one reuses with its own
        workspace, so both can run concurrently on different streams."""
        if not torch.cuda.is_available():
            raise RuntimeError("hddm needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", device)
        self.prob = prob
        self.ngx = prob.nx + 2 * prob.npml
        self.ngy = prob.ny + 2 * prob.npml
        self.ctx = H.hddm_setup(prob, velocity, device)
        self.restart = restart
        self.factor_bytes, self.work_bytes, self.krylov_bytes = H.hddm_query_bytes(self.ctx, restart)
        self.factor_buf = (share_from.factor_buf if share_from is not None
                           else _buf(self.factor_bytes, self.device))
        self.work_buf = _buf(self.work_bytes, self.device)
        self.krylov_buf = None
        H.hddm_bind(self.ctx, self.factor_buf.data_ptr(), self.factor_buf.numel(),
                    self.work_buf.data_ptr(), self.work_buf.numel(), _stream(self.device))
        if share_from is not None:
            H.hddm_share_factor(self.ctx, share_from.ctx)

    def factor(self):
        H.hddm_factor(self.ctx, _stream(self.device))

    def _vec(self, a):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
        a = a.to(self.device, torch.complex128).contiguous()
        assert a.numel() == self.ngx * self.ngy
        return a

    def empty(self):
        return torch.empty((self.ngy, self.ngx), dtype=torch.complex128, device=self.device)

    def apply_precond(self, r, out=None):
        r = self._vec(r)
        z = self.empty() if out is None else out
        H.hddm_apply_precond(self.ctx, r.data_ptr(), z.data_ptr(), _stream(self.device))
        return z

    def matvec(self, x, out=None):
        x = self._vec(x)
        y = self.empty() if out is None else out
        H.hddm_matvec(self.ctx, x.data_ptr(), y.data_ptr(), _stream(self.device))
        return y

    def ensure_krylov(self, restart):
        _, _, kb = H.hddm_query_bytes(self.ctx, restart)
        if self.krylov_buf is None or self.krylov_buf.numel() < kb:
            self.krylov_buf = None
            self.krylov_buf = _buf(kb, self.device)
        return self.krylov_buf

    def solve(self, rhs, tol=1e-8, restart=None, maxit=10000, out=None, raise_on_noconv=True,
              ortho=H.ORTHO_CGS2):
        restart = self.restart if restart is None else restart
        b = self._vec(rhs)
        x = self.empty() if out is None else out
        kb = self.ensure_krylov(restart)
        opts = H.SolveOpts(tol=tol, restart=restart, maxit=maxit, ortho=ortho, reserved=0)
        info = H.hddm_solve(self.ctx, b.data_ptr(), x.data_ptr(), opts, kb.data_ptr(), kb.numel(),
                            _stream(self.device), raise_on_noconv=raise_on_noconv)
        return x, info.as_dict()

    def ddm_solve(self, rhs, max_steps=1000, tol=1e-8, out=None, raise_on_noconv=True):
        """The iterative multi-step DDM (eq. ddms) as a solver: steps of local
        solves with the neighbours' residuals as sources, summed."""
        b = self._vec(rhs)
        x = self.empty() if out is None else out
        wb = H.hddm_ddm_query_bytes(self.ctx)
        if getattr(self, "ddm_buf", None) is None or self.ddm_buf.numel() < wb:
            self.ddm_buf = None
            self.ddm_buf = _buf(wb, self.device)
        info = H.hddm_ddm_solve(self.ctx, b.data_ptr(), x.data_ptr(), max_steps, tol,
                                self.ddm_buf.data_ptr(), self.ddm_buf.numel(),
                                _stream(self.device), raise_on_noconv=raise_on_noconv)
        return x, info.as_dict()

    # ---- block form: up to 16 right-hand sides per sweep
    def _vecs(self, a):
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
        a = a.to(self.device, torch.complex128).contiguous()
        assert a.numel() % (self.ngx * self.ngy) == 0
        return a.reshape(-1, self.ngy, self.ngx)

    def ensure_block(self, nrhs, restart):
        """Block workspace and Krylov buffer for nrhs right-hand sides."""
        wb, kb = H.hddm_query_block_bytes(self.ctx, nrhs, restart)
        if getattr(self, "block_buf", None) is None or self.block_buf.numel() < wb:
            self.block_buf = None
            self.block_buf = _buf(wb, self.device)
        if getattr(self, "block_krylov", None) is None or self.block_krylov.numel() < kb:
            self.block_krylov = None
            self.block_krylov = _buf(kb, self.device)
        return self.block_buf, self.block_krylov

    def apply_precond_block(self, R, out=None):
        """z_k = P^-1 r_k for the rows of R ([nrhs, ngy, ngx], nrhs <= 16)."""
        R = self._vecs(R)
        nr = R.shape[0]
        Z = torch.empty_like(R) if out is None else out
        wb, _ = self.ensure_block(nr, 1)
        n = self.ngx * self.ngy
        H.hddm_apply_precond_block(self.ctx, R.data_ptr(), n, Z.data_ptr(), n, nr, wb.data_ptr(),
                                   wb.numel(), _stream(self.device))
        return Z

    def solve_block(self, B, tol=1e-8, restart=None, maxit=10000, out=None, raise_on_noconv=True,
                    ortho=H.ORTHO_CGS2):
        """Solve for the rows of B ([nrhs, ngy, ngx], nrhs <= 16) together."""
        restart = self.restart if restart is None else restart
        B = self._vecs(B)
        nr = B.shape[0]
        X = torch.empty_like(B) if out is None else out
        wb, kb = self.ensure_block(nr, restart)
        n = self.ngx * self.ngy
        opts = H.SolveOpts(tol=tol, restart=restart, maxit=maxit, ortho=ortho, reserved=0)
        infos = H.hddm_solve_block(self.ctx, B.data_ptr(), n, X.data_ptr(), n, nr, opts,
                                   wb.data_ptr(), wb.numel(), kb.data_ptr(), kb.numel(),
                                   _stream(self.device), raise_on_noconv=raise_on_noconv)
        return X, [i.as_dict() for i in infos]

    def history(self, rhs=0):
        """Residual estimates after every Arnoldi step of the last solve
        (right-hand side `rhs` of a block solve), numpy float64."""
        return H.hddm_solve_history(self.ctx, rhs)

    def close(self):
        if self.ctx is not None:
            H.hddm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
