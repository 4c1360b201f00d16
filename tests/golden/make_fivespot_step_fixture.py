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
of the Jacobian scaled by the inverses of its diagonal blocks (D^-1 J, whose
diagonal pivots are then 1), to the oracle's relative residual of 1e-12.  The unknowns
are put in a nested-dissection order of the grid first (recursive
bisection of the box along its longest axis, each separator plane after
the two halves it splits, the wells last), which SuperLU factors about four
times faster than in its own column order.  The Newton iteration, updates,
convergence tests and time-step control are the oracle's.  Run from the
repository root (about 4.5 minutes per Newton iteration, 10 GB of memory;
the step takes more than 24 Newton iterations, the oracle cutting it once):

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


def nested_dissection(nx, ny, nz, leaf=256):
    """Cells of an nx x ny x nz grid in nested-dissection order: a box of at
    most `leaf` cells in natural order, a larger one split at the middle plane
    of its longest axis, the two halves first and the plane after them."""
    out = []

    def rec(lo, hi):
        ext = [h - l for l, h in zip(lo, hi)]
        if ext[0] * ext[1] * ext[2] <= leaf:
            for k in range(lo[2], hi[2]):
                for j in range(lo[1], hi[1]):
                    out.extend(i + nx * (j + ny * k) for i in range(lo[0], hi[0]))
            return
        a = max(range(3), key=lambda d: (ext[d], -d))     # the first longest axis
        m = (lo[a] + hi[a]) // 2
        left, right, plane = list(hi), list(lo), (list(lo), list(hi))
        left[a], right[a] = m, m + 1
        plane[0][a], plane[1][a] = m, m + 1
        rec(lo, left)
        rec(right, hi)
        rec(*plane)

    rec([0, 0, 0], [nx, ny, nz])
    return np.array(out, dtype=np.int64)


class LuGmres:
    """J x = rhs by GMRES(50) preconditioned with the SuperLU factors of J in
    nested-dissection order (the wells last), factored at every call."""

    def __init__(self, dims, rtol=1e-12, max_restarts=8):
        self.rtol, self.max_restarts = rtol, max_restarts
        self.cells = nested_dissection(*dims)
        self.lu = None
        self.perm = None
        self.fn = LINSOLVE_FN(self._call)

    def _matrix(self, nrows, nb, rowptr, colind, val):
        import scipy.sparse as sp
        rp = np.ctypeslib.as_array(rowptr, shape=(nrows + 1,)).copy()
        nnzb = int(rp[-1])
        ci = np.ctypeslib.as_array(colind, shape=(nnzb,)).copy()
        v = np.ctypeslib.as_array(val, shape=(nnzb * nb * nb,)).reshape(nnzb, nb, nb).copy()
        n = nrows * nb
        # the inverses of the diagonal blocks (one per block row), as a
        # block-diagonal matrix: the factors are those of D^-1 A, whose
        # diagonal pivots are 1
        rows = np.repeat(np.arange(nrows), np.diff(rp))
        d = v[ci == rows]
        self.dinv = sp.bsr_matrix((np.linalg.inv(d), np.arange(nrows), np.arange(nrows + 1)),
                                  shape=(n, n)).tocsr()
        return sp.bsr_matrix((v, ci, rp), shape=(n, n)).tocsc()

    def _gmres(self, A, b):
        import scipy.sparse.linalg as sla
        its = [0]

        def count(_):
            its[0] += 1
        p = self.perm
        inv = np.empty_like(p)
        inv[p] = np.arange(p.size)

        def prec(v):
            return self.lu.solve((self.dinv @ v)[p])[inv]
        M = sla.LinearOperator(A.shape, matvec=prec)
        x, info = sla.gmres(A, b, M=M, rtol=self.rtol, atol=0.0, restart=50,
                            maxiter=self.max_restarts, callback=count, callback_type="pr_norm")
        rel = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        return x, its[0], info == 0 and rel <= 10 * self.rtol

    def _call(self, ctx, nrows, nb, rowptr, colind, val, rhs, x, iters):
        try:
            import scipy.sparse.linalg as sla
            A = self._matrix(nrows, nb, rowptr, colind, val)
            b = np.ctypeslib.as_array(rhs, shape=(nrows * nb,)).copy()
            n = self.cells.size
            self.perm = np.concatenate([(self.cells[:, None] * nb + np.arange(nb)).ravel(),
                                        np.arange(n * nb, nrows * nb)])
            Ap = (self.dinv @ A.tocsr())[self.perm][:, self.perm].tocsc()
            # diagonal pivots first (the fill of the nested-dissection order,
            # no more); threshold pivoting only if GMRES does not converge
            # on those factors
            for thresh in (0.0, 0.1):
                t0 = time.time()
                self.lu = sla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=thresh,
                                   options=dict(SymmetricMode=True))
                print(f"  factored the Jacobian in {time.time() - t0:.0f} s "
                      f"(pivot threshold {thresh})", flush=True)
                xs, it, ok = self._gmres(A, b)
                if ok:
                    break
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
    solver = LuGmres(DIMS)
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
