"""Pins of the oracle's per-cell properties (PVT tables, Corey, densities,
accumulations) and of their analytic derivatives."""
import json
import math
import os

import numpy as np
import pytest

from paper_2406_10862_amd import reservoirs as rv
from oracle.fimref import OracleModel, prop_index
from tests.helpers import box, blackoil_mixed_state

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def one_cell(fluid, P, Sw, X=0.0, flag=0, cr=3e-6):
    res = box(1, 1, 1, fluid=fluid, p0=P, sw0=Sw, x0=X, flag0=flag, cr=cr)
    return OracleModel(res)


def test_table_nodes_reproduce_and_interpolate_linearly():
    fl = rv.deadoil_fluid()
    ix = prop_index(2)
    for r in [0, 3, 10, 18]:
        m = one_cell(fl, fl.p[r], 0.5)
        pr = m.props()
        assert 1.0 / pr[ix["b_o"], 0] == pytest.approx(fl.bo[r], rel=1e-15)
    # midpoint of an interval: B is the mean of the two node values
    p_mid = 0.5 * (fl.p[6] + fl.p[7])
    b = one_cell(fl, p_mid, 0.5).props()[ix["b_o"], 0]
    assert 1.0 / b == pytest.approx(0.5 * (fl.bo[6] + fl.bo[7]), rel=1e-15)
    # below the first node the first interval extrapolates linearly
    slope = (fl.bo[1] - fl.bo[0]) / (fl.p[1] - fl.p[0])
    b = one_cell(fl, 100.0, 0.5).props()[ix["b_o"], 0]
    assert 1.0 / b == pytest.approx(fl.bo[0] + slope * (100.0 - fl.p[0]), rel=1e-14)


def test_water_compressibility_definition():
    fl = rv.deadoil_fluid()
    ix = prop_index(2)
    b1 = one_cell(fl, 3000.0, 0.5).props()[ix["b_w"], 0]
    b2 = one_cell(fl, 5000.0, 0.5).props()[ix["b_w"], 0]
    # c_w = d ln b_w / dP is constant
    assert math.log(b2 / b1) / 2000.0 == pytest.approx(fl.cw, rel=1e-9)
    b_ref = one_cell(fl, fl.pw_ref, 0.5).props()[ix["b_w"], 0]
    assert b_ref == pytest.approx(1.0 / fl.bw_ref, rel=1e-15)


def test_corey_quadratic_half_and_clamps():
    fl = rv.deadoil_fluid(swc=0.2, sor=0.2)
    ix = prop_index(2)
    half = GOLD["corey_quadratic_at_half"]["value"]
    # normalised water saturation 0.5 -> Sw = 0.2 + 0.5*0.6 = 0.5
    pr = one_cell(fl, 4700.0, 0.5).props()[:, 0]
    krw = pr[ix["Lam_w"]] * fl.muw / pr[ix["b_w"]]
    kro = pr[ix["Lam_o"]] * 2.0 / pr[ix["b_o"]]
    assert krw == pytest.approx(half * fl.krw_max, rel=1e-14)
    assert kro == pytest.approx(half * fl.kro_max, rel=1e-14)
    # below connate water: water immobile, zero derivative
    pr = one_cell(fl, 4700.0, 0.1).props()[:, 0]
    assert pr[ix["Lam_w"]] == 0.0 and pr[ix["dLam_w_dSw"]] == 0.0
    # above 1 - Sor: oil immobile, water at its end point
    pr = one_cell(fl, 4700.0, 0.9).props()[:, 0]
    assert pr[ix["Lam_o"]] == 0.0
    assert pr[ix["Lam_w"]] * fl.muw / pr[ix["b_w"]] == pytest.approx(fl.krw_max)


def test_surface_density_and_oil_mass_identity():
    # a fluid at unit formation volume factors has its stock-tank densities
    p = rv.table_pressures()
    fl = rv.Fluid(model=2, p=p, bo=np.ones_like(p), rs=np.zeros_like(p),
                  muo=np.ones_like(p), bg=np.ones_like(p), mug=np.ones_like(p),
                  bw_ref=1.0, cw=0.0, pw_ref=14.7)
    ix = prop_index(2)
    pr = one_cell(fl, 3000.0, 0.5).props()[:, 0]
    assert pr[ix["gam_w"]] * 144.0 == pytest.approx(fl.rho_sc[0], rel=1e-15)
    assert pr[ix["gam_o"]] * 144.0 == pytest.approx(fl.rho_sc[1], rel=1e-15)
    # saturated black oil: the mass in one reservoir barrel of oil equals one
    # stock-tank barrel of oil plus Rs Mscf of dissolved gas, divided by Bo
    fl3 = rv.blackoil_fluid()
    ix3 = prop_index(3)
    P = 3700.0
    pr = one_cell(fl3, P, 0.3, X=0.1, flag=rv.SAT).props()[:, 0]
    rs = np.interp(P, fl3.p, fl3.rs)
    bo_res = 1.0 / pr[ix3["b_o"]]
    mass = fl3.rho_sc[1] * 5.615 + rs * fl3.rho_sc[2]
    assert pr[ix3["gam_o"]] * 144.0 * 5.615 * bo_res == pytest.approx(mass, rel=1e-14)
    bg_res = 1.0 / pr[ix3["b_g"]]
    assert pr[ix3["gam_g"]] * 144.0 * 5.615 * bg_res == pytest.approx(fl3.rho_sc[2], rel=1e-14)


def test_saturations_sum_to_one_from_accumulations():
    # N_i = PV sum_j S_j b_j x_ij and sum_j S_j = 1 (the paper's constraints)
    res = rv.config_c1()
    rng = np.random.default_rng(7)
    P, Sw, X, flag = blackoil_mixed_state(res, rng)
    m = OracleModel(res)
    pr = m.props(P=P, Sw=Sw, X=X, flag=flag)
    ix = prop_index(3)
    pv = pr[ix["PV"]]
    sw = pr[ix["A_w"]] / (pv * pr[ix["b_w"]])
    so = pr[ix["A_o"]] / (pv * pr[ix["b_o"]])
    rs = np.where(flag == rv.SAT, np.interp(P, res.fluid.p, res.fluid.rs), X)
    sg = (pr[ix["A_g"]] / pv - rs * pr[ix["A_o"]] / pv) / pr[ix["b_g"]]
    np.testing.assert_allclose(sw, Sw, rtol=1e-13)
    np.testing.assert_allclose(sw + so + sg, 1.0, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sg, np.where(flag == rv.SAT, X, 0.0), atol=1e-13)


def test_bubble_point_continuity():
    # at Rs = Rs_sat(P) the undersaturated branch meets the saturated branch
    fl = rv.blackoil_fluid()
    ix = prop_index(3)
    for P in [2250.0, 3700.0, 6100.0]:
        rs = float(np.interp(P, fl.p, fl.rs))
        a = one_cell(fl, P, 0.3, X=rs, flag=rv.UNSAT).props()[:, 0]
        b = one_cell(fl, P, 0.3, X=0.0, flag=rv.SAT).props()[:, 0]
        for key in ["b_o", "Lam_o", "Lam_og", "gam_o", "A_w", "A_o", "A_g", "lam_t"]:
            assert a[ix[key]] == pytest.approx(b[ix[key]], rel=1e-12), key


def fd_props(m, state, nb, h_rel=1e-7):
    """Central finite differences of every property w.r.t. each unknown."""
    P, Sw, X, flag = state
    base = m.props(P=P, Sw=Sw, X=X, flag=flag)
    grads = []
    for u, arr in enumerate([P, Sw, X][:nb]):
        h = h_rel * np.maximum(np.abs(arr), 1.0 if u == 0 else 0.1)
        up = [P.copy(), Sw.copy(), X.copy()]
        dn = [P.copy(), Sw.copy(), X.copy()]
        up[u] = arr + h
        dn[u] = arr - h
        pu = m.props(P=up[0], Sw=up[1], X=up[2], flag=flag)
        pd = m.props(P=dn[0], Sw=dn[1], X=dn[2], flag=flag)
        grads.append((pu - pd) / (2 * h))
    return base, grads


@pytest.mark.parametrize("cfg", ["deadoil", "blackoil"])
def test_property_derivatives_match_finite_differences(cfg):
    rng = np.random.default_rng(11)
    if cfg == "deadoil":
        res = rv.config_c2_small(6, 5, 3)
        n = res.n
        P = 4550.0 + 400.0 * rng.uniform(size=n)
        Sw = rng.uniform(0.25, 0.75, size=n)
        X = np.zeros(n)
        flag = np.zeros(n, np.int8)
        nb = 2
    else:
        res = rv.config_c1()
        P, Sw, X, flag = blackoil_mixed_state(res, rng)
        nb = 3
    m = OracleModel(res)
    base, grads = fd_props(m, (P, Sw, X, flag), nb)
    ix = prop_index(nb)
    names = {v: k for k, v in ix.items()}
    unk = ["P", "Sw", "X"][:nb]
    checked = 0
    for q, name in names.items():
        if "_d" in name:
            continue
        for u, un in enumerate(unk):
            key = f"d{name}_d{un}"
            if key not in ix:
                continue
            an = base[ix[key]]
            fd = grads[u][q]
            scale = np.maximum(np.abs(an), 1e-8 * np.abs(base[q]).max() + 1e-300)
            err = np.abs(an - fd) / scale
            assert err.max() < 1e-5, (key, err.max())
            checked += 1
    assert checked >= 10


def test_exact_table_node_takes_right_hand_slope():
    # reading of the table interpolation: P on a node belongs to the interval
    # that starts at that node, so the derivative is that interval's slope
    fl = rv.deadoil_fluid()
    ix = prop_index(2)
    r = 7
    pr = one_cell(fl, fl.p[r], 0.5).props()[:, 0]
    b = pr[ix["b_o"]]
    slope_B = (fl.bo[r + 1] - fl.bo[r]) / (fl.p[r + 1] - fl.p[r])
    # A_o = PV b_o So: d/dP at fixed So holds PV' b + PV b', with b' = -B'/B^2
    pv = pr[ix["PV"]]
    so = 0.5
    dpv = pv / (1 + 3e-6 * (fl.p[r] - 4700.0)) * 3e-6
    expect = dpv * b * so + pv * (-slope_B * b * b) * so
    assert pr[ix["dA_o_dP"]] == pytest.approx(expect, rel=1e-12)
