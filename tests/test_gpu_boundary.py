"""GPU checks of the boundary and the failure paths: device-pointer state
input, non-finite and non-physical states (rollback and FIM_NOT_CONVERGED,
as the oracle does), and the large-level AMG restriction forced onto small
odd grids."""
import numpy as np
import pytest

from paper_2406_10862_amd import fim, reservoirs as rv
from oracle.fimref import OracleModel
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


@pytest.mark.parametrize("cfg", ["c2s", "c1"])
def test_set_state_dev_equals_set_state_bitwise(cfg):
    torch = _torch()
    res = rv.config_c1() if cfg == "c1" else rv.config_c2_small(9, 11, 4)
    rng = np.random.default_rng(3)
    P = res.p0 + rng.uniform(-50, 50, size=res.n)
    Sw = np.clip(res.sw0 + rng.uniform(0, 0.05, size=res.n), 0, 1)
    X = np.asarray(res.x0, np.float64).copy()
    flag = np.asarray(res.flag0, np.int8).copy()
    a = fim.Fim(res)
    a.fim_set_state(P, Sw, X, flag)
    b = fim.Fim(res)
    d = torch.device("cuda")
    t = lambda v: torch.from_numpy(np.ascontiguousarray(v)).to(d)
    b.fim_set_state_dev(t(P), t(Sw), t(X), t(flag))
    sa, sb = a.fim_get_state(), b.fim_get_state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    # and the step-start accumulation it recorded: one step from each is the same
    ra, rb = a.fim_step(res.schedule[0]), b.fim_step(res.schedule[0])
    assert ra[0] == rb[0] == fim.FIM_OK
    sa, sb = a.fim_get_state(), b.fim_get_state()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k


def test_set_state_dev_rejects_tensors_of_the_wrong_shape_or_type():
    torch = _torch()
    res = rv.config_c2_small(5, 4, 3)
    g = fim.Fim(res)
    d = torch.device("cuda")
    n = res.n
    ok = torch.ones(n, dtype=torch.float64, device=d)
    with pytest.raises(fim.FimError, match="dtype"):
        g.fim_set_state_dev(ok.float(), ok)
    with pytest.raises(fim.FimError, match="elements"):
        g.fim_set_state_dev(ok, ok[:-1])
    with pytest.raises(fim.FimError, match="GPU tensor"):
        g.fim_set_state_dev(ok.cpu(), ok)
    with pytest.raises(fim.FimError, match="flag: dtype"):
        g.fim_set_state_dev(ok, ok, None, torch.zeros(n, dtype=torch.int32, device=d))


def _inject_and_step(res, cell, key, value, max_cuts=2):
    g, o = pair(res, options=rv.Options(max_cuts=max_cuts))
    st = dict(P=o.P.copy(), Sw=o.Sw.copy(), X=o.X.copy(), flag=o.flag.copy())
    st[key][cell] = value
    g.fim_set_state(st["P"], st["Sw"], st["X"], st["flag"], o.pbhp)
    o.set_state(st["P"], st["Sw"], st["X"], st["flag"])
    before = g.fim_get_state()
    rc, rep = g.fim_step(res.schedule[0])
    ost, orep = o.step(res.schedule[0], o.options(max_cuts=max_cuts))
    return g, before, rc, rep, ost, orep


@pytest.mark.parametrize("cfg", ["c2s", "c1"])
def test_nan_state_fails_every_cut_and_is_restored(cfg):
    res = rv.config_c1() if cfg == "c1" else rv.config_c2_small(6, 6, 3)
    g, before, rc, rep, ost, orep = _inject_and_step(res, 17, "P", np.nan)
    assert ost == 1 and orep.cuts == 3
    assert rc == fim.FIM_NOT_CONVERGED and rep.cuts == 3 and rep.converged == 0
    assert rep.nsub == 0 and rep.newton_iters == 0
    after = g.fim_get_state()
    for k in before:
        assert np.array_equal(before[k], after[k], equal_nan=True), k
    assert np.isnan(after["P"][17])


@pytest.mark.parametrize("cfg", ["c2s", "c1"])
def test_negative_saturation_state_is_rejected_like_the_oracle(cfg):
    res = rv.config_c1() if cfg == "c1" else rv.config_c2_small(6, 6, 3)
    g, before, rc, rep, ost, orep = _inject_and_step(res, 11, "Sw", -0.05)
    assert ost == 1 and orep.cuts == 3
    assert rc == fim.FIM_NOT_CONVERGED and rep.cuts == 3 and rep.nsub == 0
    assert rep.newton_iters > 0
    after = g.fim_get_state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k


@pytest.mark.parametrize("dims", [(31, 29, 7), (131, 9, 5), (67, 3, 3), (1, 40, 9)])
@pytest.mark.parametrize("cycle", [0, 2])
def test_row_segment_restriction_equals_the_lane_restriction(dims, cycle):
    """The restriction by row segments, which the library takes only on
    levels with 2^18 or more cells per colour, forced onto every level of
    small grids with odd and even extents, partial segments and coarse rows
    longer than one segment: the preconditioner's output is the same bit for
    bit as with the eight-lane restriction."""
    res = rv.config_c2_small(*dims)
    g = fim.Fim(res)
    g.set_initial_state()
    R, *_ = g.fim_assemble(10.0)
    v = np.random.default_rng(sum(dims)).normal(size=len(R))
    outs = {}
    for seg in (-1, 1, 64):
        g.fim_set_options(rv.Options(amg_cycle=cycle, amg_seg_rows=seg))
        g.fim_assemble(10.0)
        outs[seg] = g.fim_precond_apply(v)
    assert np.all(np.isfinite(outs[-1]))
    for seg, z in outs.items():
        assert np.array_equal(z, outs[-1]), seg


def test_row_segment_restriction_in_full_steps_matches_the_oracle():
    res = rv.config_c2_small(31, 29, 7, nsteps=2)
    g, o = pair(res, options=rv.Options(amg_seg_rows=1))
    for s, dt in enumerate(res.schedule):
        st, orep = o.step(dt)
        assert st == 0
        for h in orep.dt_sub[: orep.nsub]:
            assert g.fim_step(h)[0] == fim.FIM_OK
    gs = g.fim_get_state()
    assert np.abs(gs["P"] - o.P).max() / np.abs(o.P).max() <= 1e-9
    assert np.abs(gs["Sw"] - o.Sw).max() <= 1e-9
