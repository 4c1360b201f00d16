"""Pins of the oracle's linear algebra against NumPy/LAPACK and against
properties that single out block ILU(0)."""
import numpy as np
import pytest

from paper_2406_10862_amd import reservoirs as rv
from oracle import fimref as fr


@pytest.fixture(scope="module")
def jac_c2s():
    res = rv.config_c2_small(8, 9, 4)
    m = fr.OracleModel(res)
    R, val = m.assemble(dt=10.0)
    rowptr, colind = m.pattern()
    return rowptr, colind, val, R, m.nb


def test_spmv_matches_dense(jac_c2s):
    rowptr, colind, val, R, nb = jac_c2s
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    x = np.random.default_rng(0).normal(size=A.shape[0])
    y = fr.bsr_spmv(rowptr, colind, val, x, nb)
    np.testing.assert_allclose(y, A @ x, rtol=1e-12, atol=1e-14 * np.abs(A).max())


def test_block_jacobi_matches_numpy_inverse(jac_c2s):
    rowptr, colind, val, R, nb = jac_c2s
    dinv = fr.bj_setup(rowptr, colind, val, nb)
    v = val.reshape(-1, nb, nb)
    x = np.random.default_rng(1).normal(size=(len(rowptr) - 1) * nb)
    y = fr.bj_apply(dinv, x, nb)
    for r in range(len(rowptr) - 1):
        q = rowptr[r] + list(colind[rowptr[r]:rowptr[r + 1]]).index(r)
        expect = np.linalg.solve(v[q], x[r * nb:(r + 1) * nb])
        np.testing.assert_allclose(y[r * nb:(r + 1) * nb], expect, rtol=1e-10, atol=1e-300)


def _chain(nrows, nb, rng):
    """Block tridiagonal (1D chain) matrix: ILU(0) has no dropped fill."""
    rowptr = [0]
    colind = []
    for r in range(nrows):
        cols = [c for c in (r - 1, r, r + 1) if 0 <= c < nrows]
        colind += cols
        rowptr.append(len(colind))
    val = rng.normal(size=(len(colind), nb, nb))
    for r in range(nrows):
        q = rowptr[r] + colind[rowptr[r]:rowptr[r + 1]].index(r)
        val[q] += 6.0 * np.eye(nb)
    return np.array(rowptr, np.int32), np.array(colind, np.int32), val.ravel()


@pytest.mark.parametrize("nb", [2, 3])
def test_bilu0_is_exact_without_fill(nb):
    rng = np.random.default_rng(2 + nb)
    rowptr, colind, val = _chain(40, nb, rng)
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    lu = fr.bilu0(rowptr, colind, val, nb)
    b = rng.normal(size=A.shape[0])
    x = fr.bilu0_solve(rowptr, colind, lu, b, nb)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def test_bilu0_reproduces_a_on_its_pattern(jac_c2s):
    # defining property of ILU(0): (L U)_ij = A_ij for every (i, j) in the pattern
    rowptr, colind, val, R, nb = jac_c2s
    lu = fr.bilu0(rowptr, colind, val, nb).reshape(-1, nb, nb)
    nrows = len(rowptr) - 1
    L = np.eye(nrows * nb)
    U = np.zeros((nrows * nb, nrows * nb))
    for r in range(nrows):
        for q in range(rowptr[r], rowptr[r + 1]):
            c = colind[q]
            blk = lu[q]
            if c < r:
                L[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] = blk
            elif c == r:
                U[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] = np.linalg.inv(blk)
            else:
                U[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] = blk
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    LU = L @ U
    mask = np.zeros_like(A, dtype=bool)
    for r in range(nrows):
        for q in range(rowptr[r], rowptr[r + 1]):
            c = colind[q]
            mask[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] = True
    scale = np.abs(A).max(axis=1, keepdims=True)
    err = np.abs(LU - A) / scale
    assert err[mask].max() < 1e-11


def test_gmres_bilu0_matches_lapack(jac_c2s):
    rowptr, colind, val, R, nb = jac_c2s
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    xd = np.linalg.solve(A, -R)
    x, st, it, rr = fr.gmres_bilu0(rowptr, colind, val, -R, nb, rtol=1e-12)
    assert st == 0 and rr <= 1e-12
    assert np.abs(x - xd).max() / np.abs(xd).max() < 1e-8
    assert np.linalg.norm(A @ x + R) / np.linalg.norm(R) < 1e-11


def test_dense_lu_matches_lapack():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(60, 60))
    b = rng.normal(size=60)
    np.testing.assert_allclose(fr.dense_solve(A, b), np.linalg.solve(A, b), rtol=1e-9)


def test_gmres_zero_rhs_returns_zero(jac_c2s):
    rowptr, colind, val, R, nb = jac_c2s
    x, st, it, rr = fr.gmres_bilu0(rowptr, colind, val, np.zeros_like(R), nb)
    assert st == 0 and it == 0 and np.all(x == 0)
