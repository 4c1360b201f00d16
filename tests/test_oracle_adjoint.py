"""Pins of the oracle's discrete adjoint (oracle/adjoint.py): the gradient
it returns against central differences of the objective itself, and its
theta-derivative of the residual against differences of the residual."""
import copy

import numpy as np
import pytest

from oracle.adjoint import AdjointOracle
from oracle.fimref import OracleModel
from paper_2406_10862_amd import reservoirs as rv


def _scaled(res, dtheta):
    """The same reservoir with kx, ky, kz of every cell times exp(dtheta)."""
    r2 = copy.deepcopy(res)
    f = np.exp(dtheta)
    r2.kx, r2.ky, r2.kz = res.kx * f, res.ky * f, res.kz * f
    return r2


def _fd_check(res, dts, qobs, cells, h=1e-3, tol=1e-5):
    J, g = AdjointOracle(res).gradient(dts, qobs)
    assert J > 0
    for c in cells:
        d = np.zeros(len(g))
        d[c] = h
        fd = (AdjointOracle(_scaled(res, d)).objective(dts, qobs)
              - AdjointOracle(_scaled(res, -d)).objective(dts, qobs)) / (2 * h)
        assert abs(g[c] - fd) <= tol * abs(fd) + 1e-9 * np.abs(g).max(), (c, g[c], fd)


def test_gradient_matches_central_differences_two_phase():
    res = rv.config_c5(8, 7, 3)
    qobs = np.random.default_rng(1).uniform(0.0, 50.0, size=(3, len(res.wells)))
    _fd_check(res, res.schedule[:3], qobs, cells=[0, 5, 17, 40, 100, 150])


def test_gradient_matches_central_differences_three_phase():
    # gas injection: cells switch from undersaturated to saturated on the way
    res = rv.config_c1()
    qobs = np.random.default_rng(2).uniform(0.0, 2000.0, size=(3, len(res.wells)))
    _fd_check(res, res.schedule[:3], qobs, cells=[1, 11, 150, 299])


@pytest.mark.parametrize("cfg", ["c5", "c1"])
def test_theta_derivative_of_the_residual(cfg):
    """lam^T dR/dtheta_c at a fixed state against central differences of
    lam^T R with the permeability of cell c scaled (R is smooth in theta)."""
    res = rv.config_c5(8, 7, 3) if cfg == "c5" else rv.config_c1()
    a = AdjointOracle(res)
    states, hsub, _ = a.forward(res.schedule[:1])
    x, xold, dt = states[-1], states[-2], hsub[-1]
    rng = np.random.default_rng(3)
    lam = rng.normal(size=(a.n + a.nw) * a.nb)
    g = a.dR_dtheta_T(x, lam)
    h = 1e-6
    for c in [0, 3, a.n // 2, a.n - 1] + list(res.wells[0].cells[:1]):
        d = np.zeros(a.n)
        d[c] = h
        vals = []
        for s in (1, -1):
            o = OracleModel(_scaled(res, s * d))
            R, _ = o.assemble(dt, o.accum(**xold), jacobian=False, **x)
            vals.append(lam @ R)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[c] - fd) <= 1e-6 * (abs(fd) + np.abs(g).max()), (c, g[c], fd)
