"""The oracle's linear-solver hook, used by the fixture script of the large
parity case: a step whose Newton iterations solve through the hook (GMRES
with SuperLU factors in nested-dissection order, a library primitive)
reaches the state the oracle's
own solvers reach, and a failing hook fails the step the way a failing
linear solve does (cuts, then the step-start state restored)."""
import ctypes as C

import numpy as np

from oracle.fimref import LINSOLVE_FN, OracleModel
from paper_2406_10862_amd import reservoirs as rv
from tests.golden.make_fivespot_step_fixture import LuGmres


def test_hook_solver_reaches_the_oracle_state():
    res = rv.config_c2_small(12, 20, 6, nsteps=1)
    a, b = OracleModel(res), OracleModel(res)
    st_a, rep_a = a.step(res.schedule[0], a.options())
    solver = LuGmres((res.nx, res.ny, res.nz))
    opt = b.options(dense_max=0)
    opt.linsolve = C.cast(solver.fn, C.c_void_p)
    st_b, rep_b = b.step(res.schedule[0], opt)
    assert st_a == st_b == 0 and rep_b.cuts == 0
    assert np.abs(a.P - b.P).max() <= 1e-10 * np.abs(a.P).max()
    assert np.abs(a.Sw - b.Sw).max() <= 1e-10
    assert np.abs(a.pbhp - b.pbhp).max() <= 1e-10 * np.abs(a.pbhp).max()


def test_failing_hook_cuts_and_restores():
    res = rv.config_c2_small(6, 8, 3, nsteps=1)
    o = OracleModel(res)
    start = o.state()
    calls = [0]

    def fail(ctx, nrows, nb, rowptr, colind, val, rhs, x, iters):
        calls[0] += 1
        return 1
    fn = LINSOLVE_FN(fail)
    opt = o.options(max_cuts=2)
    opt.linsolve = C.cast(fn, C.c_void_p)
    st, rep = o.step(res.schedule[0], opt)
    assert st == 1 and rep.cuts == 3 and calls[0] == 3
    for k, v in start.items():
        assert np.array_equal(o.state()[k], v), k
