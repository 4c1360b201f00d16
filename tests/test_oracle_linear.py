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


# ---------------------------------------------------------------------------
# block-Jacobi ILU(0) over box subdomains (tiles)

def _model_matrix(res):
    m = fr.OracleModel(res)
    R, val = m.assemble(dt=10.0)
    rowptr, colind = m.pattern()
    return m, rowptr, colind, val


def test_tiled_ilu0_with_single_cell_tiles_is_block_jacobi():
    # every well spans several layers, so each well row is a subdomain of
    # its own: ILU(0) of 1x1 blocks is the inverse of the diagonal block
    res = rv.config_c2_small(7, 9, 3)
    m, rowptr, colind, val = _model_matrix(res)
    tiles = fr.ilu_tiles(res.nx, res.ny, res.nz, (1, 1, 1), [w.cells for w in res.wells])
    assert len(set(tiles.tolist())) == len(rowptr) - 1
    lu = fr.bilu0_tiled(rowptr, colind, val, m.nb, tiles)
    x = np.random.default_rng(11).normal(size=(len(rowptr) - 1) * m.nb)
    y = fr.bilu0_solve(rowptr, colind, lu, x, m.nb)
    np.testing.assert_allclose(y, fr.bj_apply(fr.bj_setup(rowptr, colind, val, m.nb), x, m.nb),
                               rtol=1e-12, atol=1e-14 * np.abs(y).max())


@pytest.mark.parametrize("tile", [(1, 1, 4), (1, 3, 1)])
def test_tiled_ilu0_on_line_tiles_is_exact_per_tile(tile):
    # without wells a line-shaped subdomain has a block tridiagonal matrix,
    # where ILU(0) drops no fill: the tiled solve must equal the exact solve
    # of the subdomain-diagonal part of A
    res = rv.config_c2_small(5, 6, 4)
    res.wells = []
    m, rowptr, colind, val = _model_matrix(res)
    tiles = fr.ilu_tiles(res.nx, res.ny, res.nz, tile, [])
    lu = fr.bilu0_tiled(rowptr, colind, val, m.nb, tiles)
    nb = m.nb
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    rt = np.repeat(tiles, nb)
    Ablk = np.where(rt[:, None] == rt[None, :], A, 0.0)
    b = np.random.default_rng(12).normal(size=A.shape[0])
    x = fr.bilu0_solve(rowptr, colind, lu, b, nb)
    np.testing.assert_allclose(x, np.linalg.solve(Ablk, b), rtol=1e-10, atol=1e-12 * np.abs(x).max())


def test_tiled_ilu0_reproduces_the_tile_part_of_a():
    # (L U)_ij = A_ij on the pattern inside each subdomain, 0 across them
    res = rv.config_c2_small(6, 7, 4)
    m, rowptr, colind, val = _model_matrix(res)
    nb = m.nb
    tiles = fr.ilu_tiles(res.nx, res.ny, res.nz, (3, 4, 2), [w.cells for w in res.wells])
    lu = fr.bilu0_tiled(rowptr, colind, val, nb, tiles).reshape(-1, nb, nb)
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
    LU = L @ U
    A = fr.bsr_to_dense(rowptr, colind, val, nb)
    rt = np.repeat(tiles, nb)
    for r in range(nrows):
        for q in range(rowptr[r], rowptr[r + 1]):
            c = colind[q]
            got = LU[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb]
            want = A[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] if tiles[r] == tiles[c] else 0.0
            np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-9 * np.abs(A).max())
