"""Small hand-built reservoirs for the pin tests (inputs only)."""
import numpy as np

from paper_2406_10862_amd import reservoirs as rv


def box(nx, ny, nz, dx=100.0, dy=100.0, dz=10.0, k=100.0, kv=None, poro=0.2, wells=(),
        fluid=None, p0=4700.0, sw0=0.3, x0=0.0, flag0=0, top=8000.0, cr=3e-6):
    n = nx * ny * nz
    fl = fluid if fluid is not None else rv.deadoil_fluid()

    def arr(v, size):
        a = np.asarray(v, dtype=np.float64)
        return np.full(size, float(a)) if a.ndim == 0 else a.astype(np.float64).copy()

    kk = arr(k, n)
    return rv.Reservoir(
        name=f"box{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=arr(dx, nx), dy=arr(dy, ny),
        dz=arr(dz, nz), top=top, kx=kk.copy(), ky=kk.copy(),
        kz=arr(kv, n) if kv is not None else kk.copy(), poro=arr(poro, n), cr=cr,
        pref=4700.0, fluid=fl, wells=list(wells), p0=arr(p0, n), sw0=arr(sw0, n),
        x0=arr(x0, n), flag0=np.full(n, flag0, np.int8), schedule=[1.0])


def ramp_state(res, rng, base=4550.0, gi=2.0, gj=3.0, gk=5.0, noise=0.05):
    """Pressure ramp with well-separated face potentials (no upwind ties) and
    values away from the 500-psi table nodes."""
    nx, ny, nz = res.nx, res.ny, res.nz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = base + gi * i + gj * j + gk * k + noise * rng.uniform(-1, 1, size=(nz, ny, nx))
    return P.ravel()


def blackoil_mixed_state(res, rng):
    """Mixed SAT/UNSAT three-phase state away from every kink."""
    n = res.n
    fl = res.fluid
    P = ramp_state(res, rng, base=4550.0, gi=2.0, gj=3.0, gk=5.0)
    flag = (rng.uniform(size=n) < 0.5).astype(np.int8)
    Sw = rng.uniform(0.2, 0.5, size=n)
    Sg = rng.uniform(0.05, 0.25, size=n)
    rs_sat = np.interp(P, fl.p, fl.rs)
    frac = rng.uniform(0.55, 0.9, size=n)
    Rs = frac * rs_sat
    # keep undersaturated Rs clear of the Rs-column nodes
    for r in fl.rs:
        near = np.abs(Rs - r) < 2e-3
        Rs[near] += 5e-3
    X = np.where(flag == rv.SAT, Sg, Rs)
    return P, Sw, X, flag
