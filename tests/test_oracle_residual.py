"""Pins of the oracle's residual (Sec. 2.1 eqs. (1)-(2) discretised with
TPFA, single-point upstream weighting and backward Euler) and of its
analytic Jacobian."""
import numpy as np
import pytest

from paper_2406_10862_amd import reservoirs as rv
from oracle.fimref import OracleModel, bsr_to_dense, prop_index
from tests.helpers import box, ramp_state, blackoil_mixed_state


def test_uniform_state_single_layer_no_wells_is_zero():
    res = box(5, 4, 1, k=np.linspace(10, 900, 20), p0=4321.0, sw0=0.45)
    m = OracleModel(res)
    R, _ = m.assemble(dt=3.0)
    assert np.all(R == 0.0)


def test_hydrostatic_column_has_no_flux():
    # oil column with immobile connate water: a discretely hydrostatic oil
    # pressure profile (P_{k+1} = P_k + avg(gamma_o) dz) carries no flux
    nz = 12
    res = box(1, 1, nz, dz=np.linspace(5, 30, nz), k=200.0, kv=20.0, sw0=0.2, p0=4600.0)
    m = OracleModel(res)
    depth = m.static()["depth"]
    ix = prop_index(2)
    P = np.full(nz, 4600.0)
    for _ in range(60):           # fixed point on the face densities
        g = m.props(P=P)[ix["gam_o"]]
        newP = P.copy()
        for k in range(nz - 1):
            newP[k + 1] = newP[k] + 0.5 * (g[k] + g[k + 1]) * (depth[k + 1] - depth[k])
        P = newP
    A = m.accum(P=P)
    R, _ = m.assemble(dt=1.0, Aold=A, P=P)
    # no flow relative to a 1-psi imbalance across one face
    T = m.static()["tz"][:-1].min()
    lam = m.props(P=P)[ix["Lam_o"]].max()
    assert np.abs(R).max() < 1e-9 * T * lam


def test_gravity_drives_oil_down_in_a_uniform_column():
    res = box(1, 1, 2, dz=10.0, k=100.0, sw0=0.2, p0=4600.0)
    m = OracleModel(res)
    R, _ = m.assemble(dt=1.0)
    # top cell loses oil (positive outflow residual), bottom gains it
    assert R[0 * 2 + 1] > 0 and R[1 * 2 + 1] < 0
    assert R[0 * 2 + 1] == -R[1 * 2 + 1]


def test_interior_fluxes_conserve_mass():
    res = rv.config_c2_small(7, 6, 4)
    res.wells = []
    rng = np.random.default_rng(3)
    m = OracleModel(res)
    P = ramp_state(res, rng) + rng.normal(0, 30, res.n)
    Sw = rng.uniform(0.2, 0.8, res.n)
    A = m.accum(P=P, Sw=Sw)
    R, _ = m.assemble(dt=1.0, Aold=A, P=P, Sw=Sw)
    R = R.reshape(-1, 2)
    for i in range(2):
        assert abs(R[:, i].sum()) < 1e-12 * np.abs(R[:, i]).sum()
        assert np.abs(R[:, i]).max() > 1.0


def test_single_point_upstream_uses_the_higher_potential_cell():
    # two cells on one layer, different water saturation: water flows from the
    # higher-pressure cell and carries that cell's mobility
    res = box(2, 1, 1, dx=50.0, k=100.0)
    m = OracleModel(res)
    ix = prop_index(2)
    T = m.static()["tx"][0]
    for P, Sw in [([4800.0, 4700.0], [0.6, 0.3]), ([4700.0, 4800.0], [0.6, 0.3])]:
        P, Sw = np.array(P), np.array(Sw)
        pr = m.props(P=P, Sw=Sw)
        A = m.accum(P=P, Sw=Sw)
        R, _ = m.assemble(dt=1.0, Aold=A, P=P, Sw=Sw)
        up = 0 if P[0] > P[1] else 1
        F = T * pr[ix["Lam_w"], up] * (P[0] - P[1])
        assert R[0] == pytest.approx(F, rel=1e-14)
        assert R[2] == -R[0]


def _fd_jacobian(m, state, dt, Aold, rowptr, colind):
    P, Sw, X, flag, pbhp = state
    n, nb, nw = m.n, m.nb, m.nw
    nu = (n + nw) * nb
    J = np.zeros((nu, nu))
    cols = []
    for c in range(n):
        for u in range(nb):
            cols.append((c, u))
    for w in range(nw):
        cols.append((n + w, 0))
    for (c, u) in cols:
        st_p = [P.copy(), Sw.copy(), X.copy(), pbhp.copy()]
        st_m = [P.copy(), Sw.copy(), X.copy(), pbhp.copy()]
        if c < n:
            base = [P, Sw, X][u][c]
            h = 1e-7 * max(abs(base), 1.0 if u == 0 else 0.1)
            st_p[u][c] += h
            st_m[u][c] -= h
        else:
            base = pbhp[c - n]
            h = 1e-7 * max(abs(base), 1.0)
            st_p[3][c - n] += h
            st_m[3][c - n] -= h
        Rp, _ = m.assemble(dt, Aold=Aold, jacobian=False, P=st_p[0], Sw=st_p[1], X=st_p[2],
                           flag=flag, pbhp=st_p[3])
        Rm, _ = m.assemble(dt, Aold=Aold, jacobian=False, P=st_m[0], Sw=st_m[1], X=st_m[2],
                           flag=flag, pbhp=st_m[3])
        J[:, c * nb + u] = (Rp - Rm) / (2 * h)
    return J


def _check_jacobian(res, state, dt=5.0):
    m = OracleModel(res)
    P, Sw, X, flag, pbhp = state
    Aold = m.accum(P=P + 3.0, Sw=Sw, X=X, flag=flag)
    R, val = m.assemble(dt, Aold=Aold, P=P, Sw=Sw, X=X, flag=flag, pbhp=pbhp)
    rowptr, colind = m.pattern()
    Ja = bsr_to_dense(rowptr, colind, val, m.nb)
    Jf = _fd_jacobian(m, state, dt, Aold, rowptr, colind)
    # padding slots of the well rows are identity rows by construction
    n, nb = m.n, m.nb
    for w in range(m.nw):
        for r in range(1, nb):
            Jf[(n + w) * nb + r, (n + w) * nb + r] = 1.0
    rowscale = np.abs(Ja).max(axis=1, keepdims=True)
    err = np.abs(Ja - Jf) / rowscale
    assert err.max() < 1e-6, err.max()
    # pattern: FD finds nothing outside the canonical pattern
    mask = np.abs(Ja) > 0
    assert np.all(np.abs(Jf[~mask]) <= 1e-6 * np.broadcast_to(rowscale, Jf.shape)[~mask])


def test_jacobian_matches_finite_differences_two_phase():
    res = rv.config_c2_small(6, 7, 3)
    rng = np.random.default_rng(5)
    P = ramp_state(res, rng)
    Sw = rng.uniform(0.3, 0.7, res.n)
    X = np.zeros(res.n)
    flag = np.zeros(res.n, np.int8)
    pbhp = np.array([4900.0, 4000.0, 4000.0, 4000.0, 4000.0])
    _check_jacobian(res, (P, Sw, X, flag, pbhp))


def test_jacobian_matches_finite_differences_three_phase_mixed_flags():
    res = rv.config_c1()
    rng = np.random.default_rng(9)
    P, Sw, X, flag = blackoil_mixed_state(res, rng)
    pbhp = np.array([6000.0, 1000.0])
    _check_jacobian(res, (P, Sw, X, flag, pbhp))
