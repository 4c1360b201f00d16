"""Pins of the oracle's static precompute (volumes, depths, pore volumes,
TPFA transmissibilities, Peaceman well indices) against closed forms."""
import json
import math
import os

import numpy as np
import pytest

from paper_2406_10862_amd import reservoirs as rv
from oracle.fimref import OracleModel
from tests.helpers import box

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
DARCY = GOLD["darcy_field_constant"]["value"]
BBL = GOLD["bbl_to_ft3"]["value"]


def test_equal_cells_transmissibility_closed_form():
    # equal cells: T = 0.001127 k A / dx on every interior face, 0 at the boundary
    res = box(4, 3, 2, dx=50.0, dy=30.0, dz=8.0, k=120.0, kv=12.0)
    st = OracleModel(res).static()
    nx, ny, nz = 4, 3, 2
    tx = st["tx"].reshape(nz, ny, nx)
    ty = st["ty"].reshape(nz, ny, nx)
    tz = st["tz"].reshape(nz, ny, nx)
    np.testing.assert_allclose(tx[:, :, :-1], DARCY * 120.0 * 30.0 * 8.0 / 50.0, rtol=1e-14)
    np.testing.assert_allclose(ty[:, :-1, :], DARCY * 120.0 * 50.0 * 8.0 / 30.0, rtol=1e-14)
    np.testing.assert_allclose(tz[:-1, :, :], DARCY * 12.0 * 50.0 * 30.0 / 8.0, rtol=1e-14)
    assert np.all(tx[:, :, -1] == 0) and np.all(ty[:, -1, :] == 0) and np.all(tz[-1] == 0)


def test_transmissibility_limits_and_symmetry():
    # series conductances: swapping the two cells leaves T unchanged, scaling
    # both permeabilities scales T, and an infinitely permeable neighbour
    # leaves only the half-cell conductance of the other cell
    def t2(k1, k2, dx1=40.0, dx2=60.0):
        res = box(2, 1, 1, dx=[dx1, dx2], dy=20.0, dz=5.0, k=[k1, k2])
        return OracleModel(res).static()["tx"][0]

    a = t2(30.0, 700.0)
    b = t2(700.0, 30.0, dx1=60.0, dx2=40.0)
    assert a == pytest.approx(b, rel=1e-15)
    assert t2(3 * 30.0, 3 * 700.0) == pytest.approx(3 * a, rel=1e-14)
    half = DARCY * 30.0 * 20.0 * 5.0 / 20.0          # k A / (dx1/2)
    assert t2(30.0, 1e18) == pytest.approx(half, rel=1e-12)
    # equal permeability reduces to the centre-to-centre distance
    assert t2(50.0, 50.0) == pytest.approx(DARCY * 50.0 * 100.0 / 50.0, rel=1e-14)


def test_depth_volume_pore_volume():
    dz = [20.0, 30.0, 50.0]
    res = box(2, 2, 3, dx=[10.0, 12.0], dy=[7.0, 9.0], dz=dz, poro=0.25, top=8000.0)
    st = OracleModel(res).static()
    d = st["depth"].reshape(3, 2, 2)
    assert np.all(d[0] == 8000.0 + 10.0)
    np.testing.assert_allclose(d[1] - d[0], (20.0 + 30.0) / 2)
    np.testing.assert_allclose(d[2] - d[1], (30.0 + 50.0) / 2)
    v = st["vol"].reshape(3, 2, 2)
    assert v[2, 1, 0] == pytest.approx(10.0 * 9.0 * 50.0)
    np.testing.assert_allclose(st["pvref"], st["vol"] * 0.25 / BBL, rtol=1e-15)


def test_peaceman_square_isotropic():
    ratio = GOLD["peaceman_ro_over_dx_square_isotropic"]["value"]
    w = rv.Well(rv.PROD, rv.BHP, 1000.0, np.array([4], np.int32), rw=0.3, skin=0.0)
    res = box(3, 3, 1, dx=200.0, dy=200.0, dz=15.0, k=80.0, wells=[w])
    wi = OracleModel(res).static()["wi"][0]
    expect = DARCY * 2 * math.pi * 80.0 * 15.0 / math.log(ratio * 200.0 / 0.3)
    assert wi == pytest.approx(expect, rel=1e-12)


def test_peaceman_anisotropic_symmetry_and_skin():
    def wi(kx, ky, dx, dy, skin=0.0):
        w = rv.Well(rv.PROD, rv.BHP, 1000.0, np.array([0], np.int32), rw=0.25, skin=skin)
        res = box(1, 1, 1, dx=dx, dy=dy, dz=10.0, k=1.0, wells=[w])
        res.kx[:] = kx
        res.ky[:] = ky
        return OracleModel(res).static()["wi"][0]

    a = wi(300.0, 30.0, 100.0, 40.0)
    b = wi(30.0, 300.0, 40.0, 100.0)     # rotate the cell by 90 degrees
    assert a == pytest.approx(b, rel=1e-14)
    # a skin s adds s to the log term: 1/WI grows linearly in s
    w0, w2, w4 = wi(50.0, 50.0, 80.0, 80.0), wi(50.0, 50.0, 80.0, 80.0, 2.0), \
        wi(50.0, 50.0, 80.0, 80.0, 4.0)
    assert 1 / w4 - 1 / w2 == pytest.approx(1 / w2 - 1 / w0, rel=1e-12)


def test_explicit_well_index_passes_through():
    w = rv.Well(rv.PROD, rv.BHP, 1000.0, np.array([0, 1], np.int32), wi=np.array([3.5, 7.25]))
    res = box(2, 1, 1, wells=[w])
    np.testing.assert_array_equal(OracleModel(res).static()["wi"], [3.5, 7.25])


def test_pattern_is_canonical_seven_point_plus_wells():
    res = rv.config_c1()
    m = OracleModel(res)
    rowptr, colind = m.pattern()
    n, nw = m.n, m.nw
    assert rowptr[-1] == m.nnzb
    for r in range(n + nw):
        cols = colind[rowptr[r]:rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
        assert r in cols
    # interior 7-point count: 3 * (faces) * 2 + n diagonal + 2 per perforation + well diag
    nx, ny, nz = 10, 10, 3
    faces = (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)
    nperf = sum(len(w.cells) for w in res.wells)
    assert m.nnzb == n + 2 * faces + 2 * nperf + nw
