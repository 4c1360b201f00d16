"""fim_step_noalloc, the step that allocates no device memory: through the C
ABI it must give what fim_step gives, bit for bit, on two calls in a row,
the second on a smaller system (the static scratch array keeps the first
call's contents), and it must refuse a step whose reduction partials do
not fit the array."""
import numpy as np
import pytest

from paper_2406_10862_amd import fim, reservoirs as rv

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def _same_run(res, nsteps, options=None):
    """Advance two contexts of one reservoir, one by fim_step and one by
    fim_step_noalloc, and compare states and iteration counts after every
    step."""
    a = fim.Fim(res, options=options)
    b = fim.Fim(res, options=options)
    a.set_initial_state()
    b.set_initial_state()
    for s in range(nsteps):
        dt = res.schedule[s % len(res.schedule)]
        ra, pa = a.fim_step(dt)
        rb, pb = b.fim_step_noalloc(dt)
        assert ra == rb == fim.FIM_OK, (s, ra, rb)
        assert (pa.newton_iters, pa.linear_iters, pa.cuts) == \
            (pb.newton_iters, pb.linear_iters, pb.cuts), s
        sa, sb = a.fim_get_state(), b.fim_get_state()
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), (s, k)


def test_noalloc_step_equals_fim_step_on_two_calls_the_second_smaller():
    _same_run(rv.config_c2_small(20, 24, 6), 2)
    _same_run(rv.config_c2_small(7, 9, 3), 2)


def test_noalloc_step_three_phase_and_mixed_precision():
    _same_run(rv.config_c1(), 2)
    _same_run(rv.config_c2_small(9, 8, 4), 1, rv.Options(precision=rv.MIXED))


def test_noalloc_step_rejects_a_system_whose_partials_do_not_fit():
    # restart 40 on 417,792 vector entries: 41 * 1632 partials > 65,536
    res = rv.config_c2_small(64, 64, 51)
    g = fim.Fim(res, options=rv.Options(restart=40))
    g.set_initial_state()
    before = g.fim_get_state()
    with pytest.raises(fim.FimError, match="static array holds"):
        g.fim_step_noalloc(1.0)
    after = g.fim_get_state()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    # restart 30 fits the same system
    g.fim_set_options(rv.Options(restart=30))
    rc, rep = g.fim_step_noalloc(1.0)
    assert rc == fim.FIM_OK
