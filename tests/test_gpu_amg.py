"""GPU pins of the CPR pressure hierarchy (Sec. 5.1: a pressure stage solved
by AMG inside the block preconditioner) against the definitions, with no
oracle code involved:

* level 0 is the quasi-IMPES pressure matrix: every cell row of the
  Jacobian combined with the first row of its diagonal block's inverse
  (scaled to max |w| = 1), the pressure column of each block kept; a well
  row keeps its own (BHP) entries;
* level l + 1 is the Galerkin product P^T A_l P of level l with the
  piecewise-constant interpolation of 2 x 2 x 2 aggregates (ragged at odd
  dimensions), every well its own aggregate.

Each level is checked against the product of the level above as the GPU
holds it, so an error in one coarsening shows up at that level."""
import numpy as np
import pytest

from paper_2406_10862_amd import fim, reservoirs as rv

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def _dense_pressure(g, rowptr, colind, val, nb):
    n, nw = g.n, g.nrows - g.n
    N = n + nw
    blocks = val.reshape(-1, nb, nb)
    A = np.zeros((N, N))
    for r in range(N):
        q0, q1 = rowptr[r], rowptr[r + 1]
        if r < n:
            d = next(blocks[q] for q in range(q0, q1) if colind[q] == r)
            w = np.linalg.inv(d)[0]
            m = np.abs(w).max()
            w = w / m if np.isfinite(m) and m > 0 else np.eye(nb)[0]
            for q in range(q0, q1):
                A[r, colind[q]] += w @ blocks[q][:, 0]
        else:
            for q in range(q0, q1):
                A[r, colind[q]] += blocks[q][0, 0]
    return A


def _interp(dims_f, dims_c):
    nx, ny, nz, nw = dims_f
    cx, cy, cz, cw = dims_c
    assert cw == nw and (cx, cy, cz) == (-(-nx // 2), -(-ny // 2), -(-nz // 2))
    nf, nc = nx * ny * nz, cx * cy * cz
    P = np.zeros((nf + nw, nc + nw))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                P[i + nx * (j + ny * k), i // 2 + cx * (j // 2 + cy * (k // 2))] = 1.0
    P[nf:, nc:] = np.eye(nw)
    return P


def _case(cfg):
    if cfg == "c5":
        return rv.config_c5(13, 10, 5)          # two phases, odd x and z
    if cfg == "c3":
        return rv.config_c3(9, 7, 5)            # three phases, every dimension odd
    return rv.config_c2_small(30, 44, 12)       # a hierarchy of several levels


@pytest.mark.parametrize("exact", [4096, 0])
@pytest.mark.parametrize("cfg", ["c5", "c3", "c2"])
def test_pressure_hierarchy_is_quasi_impes_then_galerkin(cfg, exact):
    res = _case(cfg)
    g = fim.Fim(res, options=rv.Options(precond=rv.PREC_CPR_ILU0, tile=(5, 5, 3),
                                        amg_exact=exact))
    g.set_initial_state()
    dt = float(res.schedule[0])
    assert g.fim_step(dt)[0] == fim.FIM_OK      # a state away from the initial one
    _, rowptr, colind, val = g.fim_assemble(dt)
    nl = g.fim_amg_levels()
    assert nl >= 2
    A0, dims0 = g.fim_amg_level(0)
    assert dims0 == (res.nx, res.ny, res.nz, len(res.wells))
    ref = _dense_pressure(g, rowptr, colind, val, g.nb)
    scale = np.abs(ref).max()
    err = np.abs(A0 - ref).max() / scale
    print(f"{cfg}: {nl} levels; level 0 {dims0} error {err:.1e}")
    assert err <= 1e-13
    prev, dprev = A0, dims0
    for lvl in range(1, nl):
        A, dims = g.fim_amg_level(lvl)
        P = _interp(dprev, dims)
        gal = P.T @ prev @ P
        err = np.abs(A - gal).max() / np.abs(gal).max()
        print(f"  level {lvl} {dims}: Galerkin error {err:.1e}")
        assert err <= 1e-13
        # a coarse well row and column carry the sums of the fine couplings
        assert np.array_equal(A[-dims[3]:, -dims[3]:] != 0, gal[-dims[3]:, -dims[3]:] != 0)
        prev, dprev = A, dims
    # the coarsest level: densely inverted (at most 64 cells), or solved by
    # slabs (at most 4096 cells), which ends the hierarchy earlier
    assert dprev[0] * dprev[1] * dprev[2] <= (64 if exact <= 0 else exact)


@pytest.mark.parametrize("cfg", ["c5", "c3", "c2"])
def test_coarse_solve_is_exact(cfg):
    """The coarsest level's solve against LAPACK on the level's dense
    operator: a slab-solved level (amg_exact) by its dense inverse from the
    slab factors applied device-wide (mode 0) and by substitution over the
    slabs (mode 1), and the default coarsest level by its dense inverse."""
    res = _case(cfg)
    out = {}
    for exact, mode in ((4096, 0), (4096, 1), (0, 0)):
        g = fim.Fim(res, options=rv.Options(precond=rv.PREC_CPR_ILU0, tile=(5, 5, 3),
                                            amg_exact=exact, amg_exact_mode=mode))
        g.set_initial_state()
        dt = float(res.schedule[0])
        assert g.fim_step(dt)[0] == fim.FIM_OK
        g.fim_assemble(dt)
        nl = g.fim_amg_levels()
        A, dims = g.fim_amg_level(nl - 1)
        b = np.random.default_rng(3).standard_normal(A.shape[0])
        x = g.fim_amg_coarse_solve(b)
        ref = np.linalg.solve(A, b)
        err = np.abs(x - ref).max() / np.abs(ref).max()
        res_norm = np.abs(A @ x - b).max() / np.abs(b).max()
        print(f"{cfg} amg_exact={exact} mode {mode}: {nl} levels, coarsest {dims}, "
              f"error {err:.1e}, residual {res_norm:.1e}")
        assert err <= 1e-9 and res_norm <= 1e-11
        out[exact, mode] = (nl, dims)
    # the slab solve takes the place of the levels below it
    assert out[4096, 0] == out[4096, 1] and out[4096, 0][0] <= out[0, 0][0]


@pytest.mark.parametrize("dims", [(5, 5, 3), (7, 5, 3)])
def test_coarse_solve_is_exact_with_few_slabs(dims):
    """The slab-solved coarsest level at its smallest (the hierarchy stops at
    the first level of at most 64 cells, and the exact level is at least
    level 1): level 1 of a 5x5x3 five-spot is 3x3x2, three slabs (one on each
    side of the twist), of 7x5x3 it is 4x3x2, four slabs (two below the
    twist, one above); both modes against LAPACK."""
    res = rv.config_c2_small(*dims)
    for mode in (0, 1):
        g = fim.Fim(res, options=rv.Options(precond=rv.PREC_CPR_ILU0, amg_exact=4096,
                                            amg_exact_mode=mode))
        g.set_initial_state()
        dt = float(res.schedule[0])
        assert g.fim_step(dt)[0] == fim.FIM_OK
        g.fim_assemble(dt)
        assert g.fim_amg_levels() == 2
        A, lvl = g.fim_amg_level(1)
        assert max(lvl[:3]) == (dims[0] + 1) // 2
        b = np.random.default_rng(5).standard_normal(A.shape[0])
        x = g.fim_amg_coarse_solve(b)
        ref = np.linalg.solve(A, b)
        err = np.abs(x - ref).max() / np.abs(ref).max()
        print(f"{dims} mode {mode}: coarsest {lvl}, error {err:.1e}")
        assert err <= 1e-9


def test_amg_exact_is_fixed_at_creation():
    res = rv.config_c5(8, 6, 3)
    g = fim.Fim(res)
    with pytest.raises(fim.FimError, match="amg_exact"):
        g.fim_set_options(rv.Options(amg_exact=4096))
    with pytest.raises(fim.FimError, match="amg_exact_mode"):
        g.fim_set_options(rv.Options(amg_exact_mode=1))


def test_amg_level_rejects_contexts_without_cpr():
    res = rv.config_c5(8, 6, 3)
    g = fim.Fim(res, options=rv.Options(precond=rv.PREC_ILU0))
    g.set_initial_state()
    g.fim_assemble(float(res.schedule[0]))
    with pytest.raises(fim.FimError, match="AMG"):
        g.fim_amg_level(0)
