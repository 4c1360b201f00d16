"""GPU checks of the batched ensemble's autotuner (fim_ensemble_tune): the
trials leave every member's state as it was, the choice is one of the
candidates, it is cached and reused, and the tuned members still compute
bit for bit what they compute alone with the tuned box, and match the
oracle."""
import os

import numpy as np
import pytest

from oracle.fimref import OracleModel
from paper_2406_10862_amd import fim, reservoirs as rv
from tests.gpu_cases import STATE_TOL, oracle_state, state_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


DIMS = [(24, 20, 12), (20, 26, 9), (30, 21, 16), (22, 22, 6)]


def _members():
    res = [rv.config_c4_member(k, d) for k, d in enumerate(DIMS)]
    members = [fim.Fim(r) for r in res]
    for m in members:
        m.set_initial_state()
    return res, members


def test_tuner_picks_a_candidate_caches_it_and_leaves_the_states(tmp_path):
    res, members = _members()
    for m in members:                      # start from the end of a first step
        assert m.fim_step(res[0].schedule[0])[0] == fim.FIM_OK
    before = [m.fim_get_state() for m in members]
    cache = str(tmp_path / "tune.txt")
    rc, rep = fim.fim_ensemble_tune(members, 15.0, trial_steps=1, cache_path=cache)
    cands = [tuple(rep.cand[c]) for c in range(rep.ncand)]
    times = [rep.trial_ms[c] for c in range(rep.ncand)]
    print("candidates", cands, "trial ms", [round(t, 1) for t in times], "chose", tuple(rep.box))
    assert rc == fim.FIM_OK and rep.from_cache == 0 and rep.trials == rep.ncand >= 2
    assert tuple(rep.box) in cands
    assert times[cands.index(tuple(rep.box))] == min(times)
    for m, b in zip(members, before):
        a = m.fim_get_state()
        for k in a:
            assert np.array_equal(a[k], b[k]), k
    text = open(cache).read().split()
    assert text[1:4] == [str(v) for v in rep.box]
    # the same key again: the cached box, no trials
    rc, rep2 = fim.fim_ensemble_tune(members, 15.0, trial_steps=1, cache_path=cache)
    assert rc == fim.FIM_OK and rep2.from_cache == 1 and rep2.trials == 0
    assert tuple(rep2.box) == tuple(rep.box)


def test_tuned_members_equal_their_lone_runs_and_the_oracle(tmp_path):
    res, members = _members()
    rc, rep = fim.fim_ensemble_tune(members, 15.0, trial_steps=1,
                                    cache_path=str(tmp_path / "tune.txt"))
    assert rc == fim.FIM_OK
    box = tuple(rep.box)
    nsteps = 2
    dt = np.array([r.schedule[:nsteps] for r in res])
    rc, status, reps = fim.fim_ensemble_run(members, dt)
    assert rc == fim.FIM_OK and np.all(status == fim.FIM_OK)
    for k, r in enumerate(res):
        alone = fim.Fim(r, options=rv.Options(tile=box))
        alone.set_initial_state()
        for s in range(nsteps):
            rc1, rep1 = alone.fim_step(dt[k, s])
            assert rc1 == fim.FIM_OK
            assert (rep1.newton_iters, rep1.linear_iters) == \
                (reps[k][s].newton_iters, reps[k][s].linear_iters)
        a, b = alone.fim_get_state(), members[k].fim_get_state()
        for q in a:
            assert np.array_equal(a[q], b[q]), (k, q)
        o = OracleModel(r)
        for s in range(nsteps):
            st, orep = o.step(dt[k, s])
            assert st == 0 and orep.cuts == 0 and reps[k][s].cuts == 0
        e = state_errors(b, oracle_state(o), r.fluid, 2)
        assert all(v <= STATE_TOL for v in e.values()), (k, e)
