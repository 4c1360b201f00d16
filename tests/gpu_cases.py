"""Shared helpers of the GPU parity tests (GPU result vs the FP64 oracle)."""
import numpy as np

from paper_2406_10862_amd import fim, reservoirs as rv
from oracle.fimref import OracleModel

# parity bar for converged states (relative to max |P|, absolute on
# saturations; Rs relative like pressure)
STATE_TOL = 1e-9


def pair(res, options=None):
    """A GPU context and an oracle model on the same reservoir and state."""
    g = fim.Fim(res, options=options)
    o = OracleModel(res)
    g.fim_set_state(o.P, o.Sw, o.X, o.flag, o.pbhp)
    return g, o


def sg_rs(state, fluid):
    sat = state["flag"] == rv.SAT
    sg = np.where(sat, state["X"], 0.0)
    rs = np.where(sat, np.interp(state["P"], fluid.p, fluid.rs), state["X"])
    return sg, rs


def state_errors(gs, os_, fluid, nb):
    eP = np.abs(gs["P"] - os_["P"]).max() / np.abs(os_["P"]).max()
    eS = np.abs(gs["Sw"] - os_["Sw"]).max()
    out = {"P": eP, "Sw": eS}
    if nb == 3:
        sg_g, rs_g = sg_rs(gs, fluid)
        sg_o, rs_o = sg_rs(os_, fluid)
        out["Sg"] = np.abs(sg_g - sg_o).max()
        out["Rs"] = np.abs(rs_g - rs_o).max() / max(np.abs(rs_o).max(), 1e-300)
    if len(os_["pbhp"]):
        out["bhp"] = np.abs(gs["pbhp"] - os_["pbhp"]).max() / np.abs(os_["pbhp"]).max()
    return out


def oracle_state(o):
    return dict(P=o.P.copy(), Sw=o.Sw.copy(), X=o.X.copy(), flag=o.flag.copy(),
                pbhp=o.pbhp.copy())


def run_parity_steps(res, nsteps, options=None):
    """Advance both sides step by step; the GPU replays the oracle's accepted
    sub-steps so both solve the same sequence of backward-Euler systems."""
    g, o = pair(res, options)
    errs = []
    for s in range(nsteps):
        dt = res.schedule[s]
        st, rep = o.step(dt)
        assert st == 0, f"oracle failed at step {s}"
        subs = list(rep.dt_sub[: rep.nsub])
        for h in subs:
            rc, grep = g.fim_step(h)
            assert rc == fim.FIM_OK, f"GPU did not converge at step {s} (dt {h})"
            assert grep.cuts == 0, f"GPU needed {grep.cuts} cuts at step {s}"
        e = state_errors(g.fim_get_state(), oracle_state(o), res.fluid, res.nb)
        errs.append(e)
        gs = g.fim_get_state()
        assert np.array_equal(gs["flag"], o.flag), f"phase flags differ at step {s}"
    return g, o, errs


def rowwise_rel_err(a, b, nb, row_scale):
    """max |a - b| / scale per block row (scale from the reference)."""
    d = np.abs(a - b).reshape(-1, nb)
    return (d.max(axis=1) / row_scale).max()
