"""GPU checks of the differentiation path: the torch.autograd binding of the
discrete adjoint against the oracle's adjoint and against central
differences of the forward objective, checkpointing every k steps against
keeping every state, and the permeability setter it relies on."""
import numpy as np
import pytest

from paper_2406_10862_amd import fim, reservoirs as rv
from tests.gpu_cases import pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def _torch():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    return torch


def _case(nsteps=4):
    res = rv.config_c5(12, 10, 4)
    res.schedule = [30.0] * 8
    qobs = np.random.default_rng(11).uniform(0.0, 60.0, size=(nsteps, len(res.wells)))
    return res, res.schedule[:nsteps], qobs


def _other_perm(res):
    """The same reservoir with the permeability field of another seed
    (porosity, wells and everything else unchanged)."""
    src = rv.config_c5(res.nx, res.ny, res.nz, seed=7)
    other = res.copy()
    other.kx, other.ky, other.kz = src.kx.copy(), src.ky.copy(), src.kz.copy()
    return other


def test_set_perm_equals_a_context_created_with_that_perm():
    res = rv.config_c5(12, 10, 4)
    other = _other_perm(res)
    a = fim.Fim(res)
    a.fim_set_perm(other.kx, other.ky, other.kz)
    b = fim.Fim(other)
    sa, sb = a.fim_static(), b.fim_static()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    a.set_initial_state()
    b.set_initial_state()
    for dt in other.schedule[:2]:
        assert a.fim_step(dt)[0] == b.fim_step(dt)[0] == fim.FIM_OK
    ga, gb = a.fim_get_state(), b.fim_get_state()
    for k in ga:
        assert np.array_equal(ga[k], gb[k]), k


def test_set_perm_dev_equals_set_perm():
    torch = _torch()
    res = rv.config_c5(12, 10, 4)
    other = _other_perm(res)
    a, b = fim.Fim(res), fim.Fim(res)
    a.fim_set_perm(other.kx, other.ky, other.kz)
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v, np.float64)).cuda()
    b.fim_set_perm_dev(t(other.kx), t(other.ky), t(other.kz))
    sa, sb = a.fim_static(), b.fim_static()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    with pytest.raises(fim.FimError, match="elements"):
        b.fim_set_perm_dev(t(other.kx[:-1]), t(other.ky), t(other.kz))


@pytest.mark.parametrize("cfg", ["c5", "c1"])
def test_checkpointing_every_k_steps_gives_the_same_gradient_bit_for_bit(cfg):
    if cfg == "c5":
        res, dts, qobs = _case(7)                 # segments of 5 + 2 steps at k = 5
        ks = (1, 2, 5, 7)
    else:
        res = rv.config_c1()
        dts = res.schedule[:3]
        qobs = np.random.default_rng(12).uniform(0.0, 2000.0, size=(3, len(res.wells)))
        ks = (1, 2)
    out = {}
    for k in (0,) + ks:
        g = fim.Fim(res, options=rv.Options(tile=(5, 5, 3)))
        g.set_initial_state()
        rc, grad, rep = g.fim_adjoint_gradient(dts, qobs, checkpoint_every=k)
        assert rc == fim.FIM_OK
        out[k] = (grad, rep.objective, rep.stored_states, g.fim_get_state(), rep.substeps)
        print(f"k={k}: stored states {rep.stored_states} recompute {rep.t_recompute_ms:.1f} ms "
              f"adjoint {rep.t_adjoint_ms:.1f} ms forward {rep.t_forward_ms:.1f} ms")
    for k in ks:
        assert np.array_equal(out[k][0], out[0][0]), k
        assert out[k][1] == out[0][1], k
        for q in out[0][3]:
            assert np.array_equal(out[k][3][q], out[0][3][q]), (k, q)
    # state copies held: every sub-step state (k = 0), or the segment starts
    # and the end plus one segment's sub-step states (k >= 1, no cuts here)
    n = len(dts)
    assert all(o[4] == n for o in out.values())
    assert out[0][2] == n + 1
    for k in ks:
        assert out[k][2] == -(-n // k) + 1 + min(k, n) + 1, k


def test_autograd_gradient_matches_the_oracle_adjoint():
    torch = _torch()
    from oracle.adjoint import AdjointOracle
    from paper_2406_10862_amd.autograd import MismatchObjective
    res, dts, qobs = _case(6)
    Jo, go = AdjointOracle(res).gradient(dts, qobs)
    obj = MismatchObjective(res, dts, qobs, options=rv.Options(tile=(5, 5, 3)),
                            checkpoint_every=5)
    theta = obj.theta0().requires_grad_(True)
    J = obj(theta)
    J.backward()
    assert J.dtype == torch.float64 and J.dim() == 0
    assert abs(J.item() - Jo) <= 1e-10 * Jo
    g = theta.grad.cpu().numpy()
    err = np.abs(g - go).max() / np.abs(go).max()
    print("autograd gradient error relative to max |grad|:", err)
    assert err <= 1e-8
    # the chain rule through a torch expression of theta
    theta2 = obj.theta0().requires_grad_(True)
    (3.0 * obj(theta2 * 1.0)).backward()
    np.testing.assert_allclose(theta2.grad.cpu().numpy(), 3.0 * g, rtol=1e-12, atol=0)


def test_autograd_gradient_matches_central_differences():
    torch = _torch()
    from paper_2406_10862_amd.autograd import MismatchObjective
    res, dts, qobs = _case(3)
    opts = rv.Options(tile=(5, 5, 3), tol_dp=1e-10, tol_ds=1e-13, lin_rtol=1e-12, forcing=0)
    obj = MismatchObjective(res, dts, qobs, options=opts, checkpoint_every=2)
    theta = obj.theta0().requires_grad_(True)
    obj(theta).backward()
    g = theta.grad.cpu().numpy()
    h = 1e-3
    cells = np.random.default_rng(5).choice(res.n, size=4, replace=False)
    with torch.no_grad():
        for c in cells:
            e = torch.zeros_like(theta)
            e[c] = h
            d = (obj(theta.detach() + e).item() - obj(theta.detach() - e).item()) / (2 * h)
            print(f"cell {c}: adjoint {g[c]:.8e} central difference {d:.8e}")
            assert abs(g[c] - d) <= 1e-4 * max(abs(d), 1e-3 * np.abs(g).max())
