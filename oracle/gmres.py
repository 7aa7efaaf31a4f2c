"""Restarted, right-preconditioned GMRES(m) in complex128 (Sec. 3: the
preconditioner is used inside GMRES with restart and a relative tolerance).

* Arnoldi on A P^-1 with classical Gram-Schmidt applied twice (CGS2);
  modified Gram-Schmidt is available as a cross-check.
* Complex Givens rotations G = [[c, s], [-conj(s), c]] with
  rho = sqrt(|a|^2 + |b|^2), c = |a|/rho, s = (a/|a|) conj(b)/rho (c = 0, s = 1
  when a = 0), which zero the subdiagonal entry b below a.
* A cycle stops when the estimated residual |gamma_{j+1}| / ||b|| <= tol; the
  update is x <- x + P^-1 (V_j y); the true residual b - A x is recomputed and,
  if still above tol, the next cycle starts from it.
* The iteration count is the total number of Arnoldi steps (= preconditioner
  applications inside Arnoldi) over all cycles.
"""
import numpy as np


def _givens(a, b):
    if a == 0:
        return 0.0, 1.0 + 0j
    rho = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def gmres(A, Pinv, b, tol=1e-8, restart=50, maxit=10000, x0=None, ortho="cgs2",
          callback=None, cycle_callback=None):
    """A, Pinv: callables on arrays shaped like b.  Returns (x, info).
    callback(iters, est) follows every Arnoldi step; cycle_callback(x, iters,
    cycles) every cycle's end, with the updated iterate (at a cycle boundary
    the iterate is the whole state: a run started again from it with x0 takes
    the same steps)."""
    shape = b.shape
    bv = b.ravel().astype(np.complex128)
    nb = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else x0.ravel().astype(np.complex128).copy()
    if nb == 0:
        return x.reshape(shape), dict(iters=0, restarts=0, relres_true=0.0, history=[])
    Av = lambda v: A(v.reshape(shape)).ravel()
    Pv = lambda v: Pinv(v.reshape(shape)).ravel()
    history = []
    iters = 0
    cycles = 0
    r = bv - Av(x) if x0 is not None else bv.copy()
    relres = np.linalg.norm(r) / nb
    while relres > tol and iters < maxit:
        cycles += 1
        beta = np.linalg.norm(r)
        # the basis vectors as rows of one array (V[:j+1] is then a view,
        # not a copy of the list of vectors)
        V = np.empty((restart + 1, bv.size), dtype=np.complex128)
        V[0] = r / beta
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart); sn = np.zeros(restart, dtype=np.complex128)
        gamma = np.zeros(restart + 1, dtype=np.complex128)
        gamma[0] = beta
        k = 0
        for j in range(restart):
            w = Av(Pv(V[j]))
            Vm = V[:j + 1]
            if ortho == "cgs2":
                h = Vm.conj() @ w
                w = w - Vm.T @ h
                h2 = Vm.conj() @ w
                w = w - Vm.T @ h2
                h = h + h2
            else:
                h = np.zeros(j + 1, dtype=np.complex128)
                for i in range(j + 1):
                    h[i] = np.vdot(V[i], w)
                    w = w - h[i] * V[i]
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            iters += 1
            # apply previous rotations to the new column
            col = H[:j + 2, j].copy()
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -np.conj(sn[i]) * col[i] + cs[i] * col[i + 1]
                col[i] = t
            c, s = _givens(col[j], col[j + 1])
            cs[j], sn[j] = c, s
            col[j] = c * col[j] + s * col[j + 1]
            col[j + 1] = 0.0
            H[:j + 2, j] = col
            gamma[j + 1] = -np.conj(s) * gamma[j]
            gamma[j] = c * gamma[j]
            est = abs(gamma[j + 1]) / nb
            history.append(est)
            if callback is not None:
                callback(iters, est)
            k = j + 1
            if est <= tol or hn == 0 or iters >= maxit:
                break
            V[j + 1] = w / hn
        R = np.triu(H[:k, :k])
        y = np.linalg.solve(R, gamma[:k])
        Vm = V[:k]
        x = x + Pv(Vm.T @ y)
        r = bv - Av(x)
        relres = np.linalg.norm(r) / nb
        if cycle_callback is not None:
            cycle_callback(x.reshape(shape), iters, cycles)
    return x.reshape(shape), dict(iters=iters, restarts=cycles, relres_true=relres, history=history)


def solve(prob, f, tol=1e-8, restart=50, maxit=10000, precond=None):
    """DDM-preconditioned GMRES on the global PML system (x0 = 0)."""
    from .operator import matvec
    from .ddm import OneStepDDM
    P = OneStepDDM(prob) if precond is None else precond
    return gmres(lambda u: matvec(prob, u), P.apply, f, tol=tol, restart=restart, maxit=maxit)
