"""The one-step DDM preconditioner (Sec. 2, eq. ddm0 and eq. pc) with its
local problems spread over a pool of worker processes.

TEST INFRASTRUCTURE ONLY, like the rest of this package.

The arithmetic is that of `ddm.OneStepDDM`, unchanged: each worker holds the
SuperLU factors of a share of the boxes (box i goes to worker i mod W); for an
application it restricts the shared residual to each of its tiles, solves the
box's local problem and writes the local solution into shared memory.  The
parent then sums all local solutions over their whole boxes, layer included,
in the lexicographic box order of `OneStepDDM.apply`.  With the same SuperLU
options the two give bitwise equal results (pinned by a test) when both
factor with one BLAS thread, as the workers do (SuperLU's supernodal updates
call BLAS, whose threaded kernels split sums differently: a multi-threaded
serial factor can differ in the last bits); only the local solves run side by
side.  `apply_many` applies the same operator to several
residuals at once: each box's SuperLU factor solves all of their local
sources as the columns of one right-hand-side matrix (one pass over the
factor), and the sums follow per residual; each result is bitwise the single
`apply` of that residual (pinned by a test).  Used where the serial form is
too slow: the large workloads' golden values and the benchmark's CPU
baseline.
"""
import multiprocessing as mp
import os
import time
from multiprocessing import shared_memory

import numpy as np

from .ddm import local_factor, restrict, smoothing
from .geometry import boxes


def _worker(prob, ids, splu_options, r_name, loc_name, shape, offsets, total, cols, conn):
    # one BLAS thread per worker: SuperLU's supernodal updates call BLAS, and
    # W workers with a full thread pool each would oversubscribe the host
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    shm_r = shared_memory.SharedMemory(name=r_name)
    shm_l = shared_memory.SharedMemory(name=loc_name)
    try:
        r = np.ndarray((cols,) + shape, dtype=np.complex128, buffer=shm_r.buf)
        loc = np.ndarray((cols, total), dtype=np.complex128, buffer=shm_l.buf)
        bxs = boxes(prob)
        t0 = time.perf_counter()
        lu = {i: local_factor(prob, bxs[i], splu_options) for i in ids}
        conn.send(("ready", time.perf_counter() - t0))
        while True:
            msg = conn.recv()
            if not (isinstance(msg, tuple) and msg[0] == "apply"):
                break
            m = msg[1]
            t0 = time.perf_counter()
            for i in ids:
                if m == 1:
                    u = lu[i].solve(restrict(r[0], bxs[i]).ravel())
                    loc[0, offsets[i]:offsets[i] + u.size] = u
                else:
                    # the m local sources as the columns of one matrix
                    B = np.stack([restrict(r[c], bxs[i]).ravel() for c in range(m)], axis=1)
                    U = lu[i].solve(B)
                    loc[:m, offsets[i]:offsets[i] + U.shape[0]] = U.T
            conn.send(("done", time.perf_counter() - t0))
        del r, loc
    finally:
        shm_r.close()
        shm_l.close()


class PooledOneStepDDM:
    """Same interface as `ddm.OneStepDDM.apply`; call `close()` (or use it as
    a context manager) to stop the workers and free the shared memory."""

    def __init__(self, prob, workers=None, smooth=False, splu_options=None, columns=1):
        """columns: the most residuals one `apply_many` call takes."""
        self.prob = prob
        self.columns = int(columns)
        self.smooth = smooth
        self.boxes = boxes(prob)
        nb = len(self.boxes)
        self.workers = max(1, min(nb, workers or os.cpu_count() or 1))
        self.shape = (prob.Ngy, prob.Ngx)
        sizes = [(b["bx"][1] - b["bx"][0]) * (b["by"][1] - b["by"][0]) for b in self.boxes]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        total = int(self.offsets[-1])
        item = np.dtype(np.complex128).itemsize
        c = self.columns
        self._shm_r = shared_memory.SharedMemory(create=True,
                                                 size=c * int(np.prod(self.shape)) * item)
        self._shm_l = shared_memory.SharedMemory(create=True, size=c * total * item)
        self._r = np.ndarray((c,) + self.shape, dtype=np.complex128, buffer=self._shm_r.buf)
        self._loc = np.ndarray((c, total), dtype=np.complex128, buffer=self._shm_l.buf)
        ctx = mp.get_context("fork")
        self._procs, self._conns = [], []
        for w in range(self.workers):
            ids = list(range(w, nb, self.workers))
            a, b = ctx.Pipe()
            p = ctx.Process(target=_worker, daemon=True,
                            args=(prob, ids, splu_options, self._shm_r.name, self._shm_l.name,
                                  self.shape, self.offsets, total, c, b))
            p.start()
            self._procs.append(p)
            self._conns.append(a)
        t = [c.recv()[1] for c in self._conns]
        self.factor_seconds_max = max(t)
        self.factor_seconds_sum = sum(t)

    def apply(self, r):
        return self.apply_many([r])[0]

    def apply_many(self, rs):
        """The preconditioner applied to each residual of the list `rs` (at
        most `columns` of them); returns the list of results."""
        m = len(rs)
        if not 1 <= m <= self.columns:
            raise ValueError(f"{m} residuals, the pool takes 1 to {self.columns}")
        for c, r in enumerate(rs):
            self._r[c] = r
        for conn in self._conns:
            conn.send(("apply", m))
        for conn in self._conns:
            conn.recv()
        out = []
        for c in range(m):
            z = np.zeros_like(rs[c], dtype=np.complex128)
            for i, box in enumerate(self.boxes):
                (bx0, bx1), (by0, by1) = box["bx"], box["by"]
                u = self._loc[c, self.offsets[i]:self.offsets[i + 1]].reshape(by1 - by0, bx1 - bx0)
                if self.smooth:
                    u = smoothing(box) * u
                z[by0:by1, bx0:bx1] += u
            out.append(z)
        return out

    def close(self):
        for c in self._conns:
            try:
                c.send("stop")
            except (BrokenPipeError, OSError):
                pass
        for p in self._procs:
            p.join(timeout=30)
        self._procs, self._conns = [], []
        self._r = self._loc = None
        for s in (self._shm_r, self._shm_l):
            s.close()
            s.unlink()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
