"""Writes the expected state of a GPU parity case too large for the oracle to
run inside a test: the oracle's state after the first 10-day step of the
60 x 220 x 20 = 264,000-cell two-phase five-spot (the 1.1M-cell benchmark's
recipe with 20 layers: sigma-2 log-normal permeability of seed 20610862,
rate scaled by the cell count; paper Sec. 3.2.5 Newton iteration, Sec.
3.3.2 time step).

Only the oracle (oracle/) and the seeded input generator run here; nothing
comes from the HIP path.  Run from the repository root:

    OMP_NUM_THREADS=8 python tests/golden/make_fivespot_step_fixture.py

It writes tests/golden/fivespot_60x220x20_step1.npz (float64 P and Sw per
cell, the wells' BHP, the accepted sub-step lengths and the oracle's
Newton and linear iteration counts).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.fimref import OracleModel  # noqa: E402
from paper_2406_10862_amd import reservoirs as rv  # noqa: E402

DIMS = (60, 220, 20)
OUT = os.path.join(HERE, "fivespot_60x220x20_step1.npz")


def workload():
    """The reservoir of the fixture (shared with the GPU test)."""
    return rv.config_c2_small(*DIMS, nsteps=1)


def main():
    res = workload()
    o = OracleModel(res)
    opt = o.options(dense_max=0, max_lin=5000)
    t0 = time.time()
    st, rep = o.step(res.schedule[0], opt)
    wall = time.time() - t0
    if st != 0:
        raise SystemExit(f"the oracle did not converge ({rep.cuts} cuts)")
    np.savez_compressed(OUT, P=o.P, Sw=o.Sw, pbhp=o.pbhp,
                        dt_sub=np.array(rep.dt_sub[: rep.nsub]),
                        newton=np.int64(rep.newton_iters), linear=np.int64(rep.linear_iters),
                        cnv=np.array(rep.cnv[:2]), mb=np.array(rep.mb[:2]))
    print(f"{res.name}: {rep.newton_iters} Newton, {rep.linear_iters} linear iterations, "
          f"{rep.cuts} cuts, {wall:.0f} s; wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
