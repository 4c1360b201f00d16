"""Writes the expected state of a GPU parity case too large for the oracle to
run inside a test: the oracle's state after the first 10-day step of the
60 x 220 x 20 = 264,000-cell two-phase five-spot (the 1.1M-cell benchmark's
recipe with 20 layers: sigma-2 log-normal permeability of seed 20610862,
rate scaled by the cell count; paper Sec. 3.2.5 Newton iteration, Sec.
3.3.2 time step).

Only the oracle (oracle/) and the seeded input generator run here; nothing
comes from the HIP path.  The oracle's own linear solver (GMRES(50) with
natural-order BILU(0)) stalls near 1e-4 on grids this size, so its Newton
iterations solve through the oracle's linear-solver hook with a library
primitive instead: GMRES preconditioned by the sparse LU factors (SuperLU)
of a recent Jacobian, refactored when GMRES fails to converge in 400
iterations, to the oracle's relative residual of 1e-12.  The Newton
iteration, updates, convergence tests and time-step control are the
oracle's.  Run from the repository root (several hours: each refactorisation
takes about 20 minutes; about 20 GB of memory):

    OMP_NUM_THREADS=8 python tests/golden/make_fivespot_step_fixture.py

It writes tests/golden/fivespot_60x220x20_step1.npz (float64 P and Sw per
cell, the wells' BHP, the accepted sub-step lengths and the oracle's
Newton and linear iteration counts).
"""
import ctypes as C
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.fimref import LINSOLVE_FN, OracleModel  # noqa: E402
from paper_2406_10862_amd import reservoirs as rv  # noqa: E402

DIMS = (60, 220, 20)
OUT = os.path.join(HERE, "fivespot_60x220x20_step1.npz")


def workload():
    """The reservoir of the fixture (shared with the GPU test)."""
    return rv.config_c2_small(*DIMS, nsteps=1)


class LuGmres:
    """J x = rhs by GMRES(50) preconditioned with the SuperLU factors of the
    last Jacobian that was factored (a factorisation costs as much as a few
    hundred GMRES iterations here); a solve that fails within
    `max_restarts` restart cycles factors the current Jacobian and solves
    again."""

    def __init__(self, rtol=1e-12, max_restarts=8):
        self.rtol, self.max_restarts = rtol, max_restarts
        self.lu = None
        self.fn = LINSOLVE_FN(self._call)

    def _matrix(self, nrows, nb, rowptr, colind, val):
        import scipy.sparse as sp
        rp = np.ctypeslib.as_array(rowptr, shape=(nrows + 1,)).copy()
        nnzb = int(rp[-1])
        ci = np.ctypeslib.as_array(colind, shape=(nnzb,)).copy()
        v = np.ctypeslib.as_array(val, shape=(nnzb * nb * nb,)).reshape(nnzb, nb, nb).copy()
        n = nrows * nb
        return sp.bsr_matrix((v, ci, rp), shape=(n, n)).tocsc()

    def _gmres(self, A, b):
        import scipy.sparse.linalg as sla
        its = [0]

        def count(_):
            its[0] += 1
        M = sla.LinearOperator(A.shape, matvec=self.lu.solve)
        x, info = sla.gmres(A, b, M=M, rtol=self.rtol, atol=0.0, restart=50,
                            maxiter=self.max_restarts, callback=count, callback_type="pr_norm")
        rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        return x, its[0], info == 0 and rel <= 10 * self.rtol

    def _call(self, ctx, nrows, nb, rowptr, colind, val, rhs, x, iters):
        try:
            import scipy.sparse.linalg as sla
            A = self._matrix(nrows, nb, rowptr, colind, val)
            b = np.ctypeslib.as_array(rhs, shape=(nrows * nb,)).copy()
            ok = False
            if self.lu is not None:
                xs, it, ok = self._gmres(A, b)
            if not ok:
                t0 = time.time()
                self.lu = sla.splu(A, permc_spec="COLAMD")
                print(f"  factored the Jacobian in {time.time() - t0:.0f} s", flush=True)
                xs, it, ok = self._gmres(A, b)
            out = np.ctypeslib.as_array(x, shape=(nrows * nb,))
            out[:] = xs
            iters[0] = it
            print(f"  linear solve: {it} GMRES iterations, ok={ok}", flush=True)
            return 0 if ok else 1
        except Exception as e:             # a ctypes callback must not raise
            print("linear solve failed:", repr(e), flush=True)
            return 1


def main():
    res = workload()
    o = OracleModel(res)
    solver = LuGmres()
    opt = o.options(dense_max=0)
    opt.linsolve = C.cast(solver.fn, C.c_void_p)
    t0 = time.time()
    st, rep = o.step(res.schedule[0], opt)
    wall = time.time() - t0
    if st != 0:
        raise SystemExit(f"the oracle did not converge ({rep.cuts} cuts)")
    np.savez_compressed(OUT, P=o.P, Sw=o.Sw, pbhp=o.pbhp,
                        dt_sub=np.array(rep.dt_sub[: rep.nsub]),
                        newton=np.int64(rep.newton_iters), linear=np.int64(rep.linear_iters),
                        cnv=np.array(rep.cnv[:2]), mb=np.array(rep.mb[:2]))
    print(f"{res.name}: {rep.newton_iters} Newton, {rep.linear_iters} linear iterations, "
          f"{rep.cuts} cuts, {wall:.0f} s; wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
