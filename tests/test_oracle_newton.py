"""Pins of the oracle's Newton iteration and time step (Sec. 3.2.5, Sec.
3.3.2): brute-force single-cell solution, the Buckley-Leverett closed form,
global mass balance, mirror symmetry, solver-path independence, cuts and
restart determinism."""
import json
import math
import os

import numpy as np
import pytest

from paper_2406_10862_amd import reservoirs as rv
from oracle.fimref import OracleModel
from tests.helpers import box

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def bisect(f, lo, hi, iters=200):
    flo = f(lo)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo <= 1e-15 * max(abs(lo), 1.0):
            break
    return 0.5 * (lo + hi)


def test_single_cell_newton_equals_nested_bisection():
    """One cell drained by one BHP producer.  For a fixed P the water
    equation is monotone in Sw; the oil equation is then monotone in P.
    Both are solved by bisection with properties evaluated independently
    here (numpy interpolation of the table, Corey curves)."""
    fl = rv.deadoil_fluid(swc=0.2, sor=0.2)
    wi, pbhp, dt = 0.8, 3000.0, 5.0
    w = rv.Well(rv.PROD, rv.BHP, pbhp, np.array([0], np.int32), wi=np.array([wi]))
    res = box(1, 1, 1, dx=100.0, dy=100.0, dz=10.0, k=100.0, poro=0.2, fluid=fl,
              wells=[w], p0=4700.0, sw0=0.35, cr=3e-6)
    pv_ref = 100.0 * 100.0 * 10.0 * 0.2 / 5.615

    def bw(P):
        return math.exp(fl.cw * (P - fl.pw_ref)) / fl.bw_ref

    def bo(P):
        return 1.0 / float(np.interp(P, fl.p, fl.bo, left=None))

    def pv(P):
        return pv_ref * (1 + res.cr * (P - res.pref))

    def kr(s):
        s = min(max(s, 0.0), 1.0)
        return s * s

    D = 1 - fl.swc - fl.sor
    Aw0 = pv(4700.0) * bw(4700.0) * 0.35
    Ao0 = pv(4700.0) * bo(4700.0) * 0.65

    def sw_of(P):
        gw = lambda S: (pv(P) * bw(P) * S - Aw0) / dt + \
            wi * kr((S - fl.swc) / D) * bw(P) / fl.muw * (P - pbhp)
        return bisect(gw, 0.0, 1.0)

    def go(P):
        S = sw_of(P)
        return (pv(P) * bo(P) * (1 - S) - Ao0) / dt + \
            wi * kr((1 - S - fl.sor) / D) * bo(P) / 2.0 * (P - pbhp)

    P_ref = bisect(go, pbhp, 4700.0)
    Sw_ref = sw_of(P_ref)
    m = OracleModel(res)
    st, rep = m.step(dt)
    assert st == 0
    assert m.P[0] == pytest.approx(P_ref, rel=1e-11)
    assert m.Sw[0] == pytest.approx(Sw_ref, abs=1e-11)


def buckley_leverett_profile(x, t, q_rb, area, poro, swc, sor, M):
    """Exact saturation at positions x (ft) and time t (days): rarefaction
    x(S) = 5.615 q t / (phi A) * df/dSw behind a Welge shock."""
    D = 1 - swc - sor
    f = lambda s: s * s / (s * s + M * (1 - s) ** 2)
    dfds = lambda s: 2 * M * s * (1 - s) / (s * s + M * (1 - s) ** 2) ** 2
    # Welge tangent f(s) = s f'(s), found by bisection
    sf = bisect(lambda s: f(s) - s * dfds(s), 1e-6, 1 - 1e-9)
    vol = 5.615 * q_rb * t / (poro * area)
    xf = vol * dfds(sf) / D
    sw = np.full_like(x, swc)
    # invert x = vol f'(s)/D on (sf, 1) where f' is decreasing
    for k, xi in enumerate(x):
        if xi >= xf:
            continue
        s = bisect(lambda s: vol * dfds(s) / D - xi, sf, 1 - 1e-12)
        sw[k] = swc + D * s
    return sw, sf, xf


def test_buckley_leverett_shock_tangent_matches_closed_form():
    for M, key in [(1.0, "buckley_leverett_shock_sn_M1"), (4.0, "buckley_leverett_shock_sn_M4")]:
        _, sf, _ = buckley_leverett_profile(np.array([0.0]), 1.0, 1.0, 1.0, 0.2, 0.2, 0.2, M)
        assert sf == pytest.approx(GOLD[key]["value"], abs=1e-12)


@pytest.mark.slow
def test_buckley_leverett_convergence():
    errs = []
    for N in [50, 100, 200, 400]:
        res = rv.buckley_leverett_1d(N)
        m = OracleModel(res)
        for dt in res.schedule:
            st, _ = m.step(dt)
            assert st == 0
        L = 1000.0
        x = (np.arange(N) + 0.5) * L / N
        t = sum(res.schedule)
        exact, sf, xf = buckley_leverett_profile(
            x, t, res.wells[0].target, 100.0, 0.2, 0.2, 0.2, 1.0)
        errs.append(np.abs(m.Sw - exact).sum() * L / N)
        if N == 400:
            # the smeared front straddles the exact shock position
            mid = 0.5 * (0.2 + 0.2 + 0.6 * sf)
            xnum = x[np.argmax(m.Sw < mid)]
            assert abs(xnum - xf) < 3 * L / N + 0.02 * xf
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.5 * errs[0]


def _mass_balance(res, nsteps):
    m = OracleModel(res)
    nb = m.nb
    for s in range(nsteps):
        dt = res.schedule[s]
        A0 = m.accum().reshape(-1, nb).sum(axis=0)
        st, rep = m.step(dt)
        assert st == 0 and rep.nsub == 1
        A1 = m.accum().reshape(-1, nb).sum(axis=0)
        q = m.well_rates().sum(axis=0)[:nb]
        err = np.abs(A1 - A0 + dt * q) / np.abs(A1)
        assert err.max() <= 1e-12, err


def test_global_mass_balance_three_phase():
    _mass_balance(rv.config_c1(), 2)


def test_global_mass_balance_two_phase():
    _mass_balance(rv.config_c2_small(10, 12, 4, nsteps=2), 2)


def test_five_spot_mirror_symmetry():
    res = rv.five_spot(9, 9, 3, 20.0, 10.0, 2.0, sigma=0.0, seed=0, inj_rate=20.0,
                       homogeneous_k=150.0, nsteps=2)
    m = OracleModel(res)
    for dt in res.schedule:
        st, _ = m.step(dt)
        assert st == 0
    P = m.P.reshape(3, 9, 9)
    S = m.Sw.reshape(3, 9, 9)
    assert np.abs(P - P[:, :, ::-1]).max() <= 1e-10 * P.max()
    assert np.abs(P - P[:, ::-1, :]).max() <= 1e-10 * P.max()
    assert np.abs(S - S[:, :, ::-1]).max() <= 1e-10
    assert np.abs(S - S[:, ::-1, :]).max() <= 1e-10
    assert S.max() > 0.25       # water has moved


def test_dense_and_iterative_paths_agree_three_phase():
    a = OracleModel(rv.config_c1())
    b = OracleModel(rv.config_c1())
    for _ in range(2):
        sa, _ = a.step(30.0, a.options(dense_max=10**6))
        sb, rb = b.step(30.0, b.options(dense_max=0))
        assert sa == 0 and sb == 0 and rb.linear_iters > rb.newton_iters
    assert np.abs(a.P - b.P).max() <= 1e-10 * a.P.max()
    assert np.abs(a.Sw - b.Sw).max() <= 1e-10
    assert np.abs(a.X - b.X).max() <= 1e-10
    assert np.array_equal(a.flag, b.flag)


def test_phase_state_consistent_after_switching():
    res = rv.config_c1()
    m = OracleModel(res)
    for _ in range(3):
        assert m.step(30.0)[0] == 0
    sat = m.flag == rv.SAT
    assert sat.sum() > 0 and (~sat).sum() > 0
    assert np.all(m.X[sat] >= 0)
    rs_sat = np.interp(m.P, res.fluid.p, res.fluid.rs)
    assert np.all(m.X[~sat] <= rs_sat[~sat] + 1e-12)


def test_failed_newton_cuts_then_restores_start_state():
    res = rv.config_c2_small(6, 6, 3)
    m = OracleModel(res)
    start = m.state()
    st, rep = m.step(10.0, m.options(max_newton=1, max_cuts=2))
    assert st == 1 and rep.cuts == 3 and rep.converged == 0 and rep.nsub == 0
    for k, v in start.items():
        assert np.array_equal(getattr(m, k), v), k


def test_cut_substeps_sum_to_the_step():
    res = rv.config_c2_small(6, 6, 3)
    m = OracleModel(res)
    st, rep = m.step(10.0, m.options(max_newton=6))
    assert st == 0 and rep.cuts == 2 and rep.nsub == 4
    assert list(rep.dt_sub[: rep.nsub]) == [2.5] * 4


def test_restart_from_saved_state_is_bitwise_identical():
    res = rv.config_c2_small(8, 8, 3, nsteps=4)
    a = OracleModel(res)
    for dt in res.schedule:
        assert a.step(dt)[0] == 0
    b = OracleModel(res)
    for dt in res.schedule[:2]:
        assert b.step(dt)[0] == 0
    saved = b.state()
    c = OracleModel(res)
    c.set_state(**saved)
    for dt in res.schedule[2:]:
        assert c.step(dt)[0] == 0
    for k in ["P", "Sw", "X", "flag", "pbhp"]:
        assert np.array_equal(getattr(a, k), getattr(c, k)), k


def test_non_finite_state_fails_every_cut_and_is_restored():
    """A NaN in the state makes the residual non-finite: every sub-step
    fails, dt is halved up to max_cuts times, then the step fails with the
    state it started from (NaN included)."""
    res = rv.config_c2_small(6, 6, 3)
    m = OracleModel(res)
    m.P[17] = np.nan
    start = m.state()
    st, rep = m.step(10.0, m.options(max_cuts=3))
    assert st == 1 and rep.cuts == 4 and rep.nsub == 0 and rep.newton_iters == 0
    for k, v in start.items():
        assert np.array_equal(getattr(m, k), v, equal_nan=True), k


@pytest.mark.parametrize("cfg", ["deadoil", "blackoil"])
def test_negative_saturation_state_is_rejected_and_restored(cfg):
    """A state with a negative water saturation in one cell reaches a root of
    the discrete equations that keeps the negative saturation (no water can
    flow out of a cell below connate saturation); a root outside [0, 1]
    fails the sub-step, so every cut fails and the step returns with its
    start state."""
    if cfg == "deadoil":
        res = rv.config_c2_small(6, 6, 3)
    else:
        res = rv.config_c1()
    m = OracleModel(res)
    m.Sw[11] = -0.05
    start = m.state()
    st, rep = m.step(res.schedule[0], m.options(max_cuts=2))
    assert st == 1 and rep.cuts == 3 and rep.nsub == 0 and rep.newton_iters > 0
    for k, v in start.items():
        assert np.array_equal(getattr(m, k), v), k
    # the same state with the cell at zero saturation steps normally
    m2 = OracleModel(res)
    m2.Sw[11] = 0.0
    st, rep = m2.step(res.schedule[0], m2.options(max_cuts=2))
    assert st == 0
