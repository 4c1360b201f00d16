"""Seeded synthetic reservoirs: the inputs shared by the GPU path and the oracle.

This module only *generates data* (grid sizes, permeability/porosity fields,
fluid tables, well lists, initial states, schedules and solver tolerances).
It contains none of the simulation arithmetic: no properties, fluxes,
transmissibilities or well indices are computed here.

The paper states the problem as grid + rock + fluid tables + wells + initial
state (Secs. 3.2.3-3.2.4, the Bulk and AllWells descriptions), validated on
SPE-style black-oil cases (Sec. 5.2).  The SPE datasets themselves are not
used; seeded stand-ins with the same shapes are generated instead.

Units are FIELD: ft, mD, psi, days, rb, stb, Mscf, cP, lb/ft3 (gas: lb/Mscf).
Cell id is c = i + nx*(j + ny*k), 0-based, k = 0 is the top layer.
"""
from __future__ import annotations

import copy
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# model ids (equal to the block size nb)
DEADOIL_OW = 2
BLACKOIL_3P = 3

# well kinds / controls
PROD, INJ_WATER, INJ_GAS = 0, 1, 2
BHP, RATE = 0, 1

# preconditioners / precision modes (option values shared with the C ABIs)
PREC_BJ, PREC_ILU0, PREC_CPR, PREC_CPR_ILU0 = 0, 1, 2, 3
FP64, MIXED = 0, 1

# phase-state flags for the three-phase model
UNSAT, SAT = 0, 1


@dataclass
class Fluid:
    model: int
    p: np.ndarray            # table pressure column [psi], strictly increasing
    bo: np.ndarray           # saturated oil FVF [rb/stb]
    rs: np.ndarray           # saturated solution GOR [Mscf/stb]
    muo: np.ndarray          # saturated oil viscosity [cP]
    bg: np.ndarray           # gas FVF [rb/Mscf]
    mug: np.ndarray          # gas viscosity [cP]
    co_us: float = 0.0       # undersaturated oil compressibility [1/psi]
    cmu_us: float = 0.0      # undersaturated oil viscosibility [1/psi]
    bw_ref: float = 1.01
    cw: float = 3e-6
    muw: float = 0.5
    pw_ref: float = 14.7
    rho_sc: tuple = (62.4, 49.0, 60.0)   # water, oil lb/ft3; gas lb/Mscf
    swc: float = 0.2
    sor: float = 0.2
    sgc: float = 0.0
    nw: float = 2.0
    no: float = 2.0
    ng: float = 2.0
    krw_max: float = 1.0
    kro_max: float = 1.0
    krg_max: float = 1.0


@dataclass
class Well:
    kind: int
    control: int
    target: float            # psi (BHP) or stb/d | Mscf/d at surface (RATE, > 0)
    cells: np.ndarray        # int32 natural cell ids (0-based)
    wi: Optional[np.ndarray] = None   # explicit well indices, else Peaceman
    rw: float = 0.25
    skin: float = 0.0
    bhp0: Optional[float] = None      # initial BHP guess (defaults: target or P0)


@dataclass
class Options:
    tol_cnv: float = 1e-6
    tol_mb: float = 1e-12
    tol_dp: float = 1e-7
    tol_ds: float = 1e-10
    tol_well: float = 1e-6
    ds_max: float = 0.2
    dp_max: float = 1000.0
    lin_rtol: float = 1e-8
    max_newton: int = 20
    max_lin: int = 400
    restart: int = 30
    max_cuts: int = 8
    precond: int = PREC_CPR_ILU0
    precision: int = FP64
    amg_cycle: int = 0          # 0 = V at the finest level, W below; 1 = V; 2 = W; >=16 by size
    amg_sweeps: int = 1
    graphs: int = 1             # replay Arnoldi steps as HIP graphs
    forcing: int = 1            # Eisenstat-Walker forcing term (lin_rtol is the floor)
    amg_fused: int = 0          # cells below which the AMG cycle runs fused (0 default, <0 off)
    tile: tuple = (0, 0, 0)     # block-Jacobi ILU(0) subdomain box (0 = 8 cells per axis)
    amg_seg_rows: int = 0       # entries per colour from which AMG restricts by row segments
    gs_refine: int = 0          # Gram-Schmidt second pass: 1 when cancelled, -1 never, 0 default (never)
    amg_exact: int = 0          # cells of a coarsest level solved exactly by slabs (<= 0: off)
    amg_exact_mode: int = 0     # 0: its dense inverse applied device-wide; 1: slab substitution


@dataclass
class Reservoir:
    name: str
    nx: int
    ny: int
    nz: int
    dx: np.ndarray
    dy: np.ndarray
    dz: np.ndarray
    top: float
    kx: np.ndarray
    ky: np.ndarray
    kz: np.ndarray
    poro: np.ndarray
    cr: float
    pref: float
    fluid: Fluid
    wells: List[Well]
    p0: np.ndarray
    sw0: np.ndarray
    x0: np.ndarray           # Sg (flag SAT) or Rs (flag UNSAT); zeros for 2-phase
    flag0: np.ndarray        # int8
    schedule: List[float]
    options: Options = field(default_factory=Options)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nb(self) -> int:
        return self.fluid.model

    def copy(self) -> "Reservoir":
        return copy.deepcopy(self)


# ----------------------------------------------------------------------------
# building blocks


def cell_id(nx, ny, i, j, k):
    """0-based natural id of 0-based (i, j, k)."""
    return i + nx * (j + ny * k)


def column_cells(nx, ny, nz, i, j, k0=0, k1=None):
    """Cells of the vertical column (i, j) for layers k0..k1-1 (0-based)."""
    k1 = nz if k1 is None else k1
    return np.array([cell_id(nx, ny, i, j, k) for k in range(k0, k1)], dtype=np.int32)


def lognormal_perm(nx, ny, nz, sigma, seed, mean_md=100.0, smooth=5.0):
    """Seeded, spatially correlated log-normal horizontal permeability.

    z ~ N(0,1) iid, Gaussian-filtered with a 5-cell standard deviation,
    re-standardised, then ln kh = ln(mean) + sigma*z.  Returns (kh, rank
    porosity) flattened in natural order.  The porosity is
    0.1 + 0.2 * rank(ln kh)/(N-1) (ties by cell id).
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    z = rng.standard_normal((nz, ny, nx))   # [k][j][i] -> C order = natural id
    z = gaussian_filter(z, sigma=smooth, mode="reflect", truncate=4.0)
    z = (z - z.mean()) / z.std()
    lnk = np.log(mean_md) + sigma * z.ravel()
    kh = np.exp(lnk)
    n = kh.size
    order = np.argsort(lnk, kind="stable")
    rank = np.empty(n, dtype=np.float64)
    rank[order] = np.arange(n, dtype=np.float64)
    poro = 0.1 + 0.2 * rank / max(n - 1, 1)
    return kh, poro


def table_pressures(nrows=20, dp=500.0):
    return dp * (np.arange(nrows, dtype=np.float64) + 1.0)


def deadoil_fluid(swc=0.2, sor=0.2) -> Fluid:
    """Dead-oil / water fluid: Bo = 1.05 exp(-1e-5 (P-5500)) sampled on 20 rows,
    muo = 2 cP, water Bw = 1.01 exp(-3e-6 (P - 14.7)), muw = 0.5 cP."""
    p = table_pressures()
    bo = 1.05 * np.exp(-1e-5 * (p - 5500.0))
    z = np.zeros_like(p)
    return Fluid(model=DEADOIL_OW, p=p, bo=bo, rs=z.copy(), muo=np.full_like(p, 2.0),
                 bg=np.ones_like(p), mug=np.ones_like(p), swc=swc, sor=sor, sgc=0.0)


def blackoil_fluid(swc=0.12, sor=0.10) -> Fluid:
    """Generic smooth synthetic black-oil tables on 20 rows, 500..10000 psi."""
    p = table_pressures()
    rs = 0.25 * (p / 1000.0) ** 0.9
    bo = 1.0 + 0.25 * rs
    bg = 2900.0 / p
    muo = 1.5 / (1.0 + rs)
    mug = 0.012 + 4e-6 * p
    return Fluid(model=BLACKOIL_3P, p=p, bo=bo, rs=rs, muo=muo, bg=bg, mug=mug,
                 co_us=1.5e-5, cmu_us=0.0, swc=swc, sor=sor, sgc=0.0)


def rs_sat_table(fluid: Fluid, pb: float) -> float:
    """Table lookup of the saturated Rs at pb (input preparation only)."""
    return float(np.interp(pb, fluid.p, fluid.rs))


# ----------------------------------------------------------------------------
# configurations


def config_c1() -> Reservoir:
    """10x10x3 three-phase black oil (SPE1-like geometry), 3x3 blocks."""
    nx, ny, nz = 10, 10, 3
    n = nx * ny * nz
    dz_l = np.array([20.0, 30.0, 50.0])
    kh_l = np.array([500.0, 50.0, 200.0])
    kh = np.repeat(kh_l, nx * ny)
    fl = blackoil_fluid(swc=0.12, sor=0.10)
    rs0 = rs_sat_table(fl, 4000.0)
    wells = [
        Well(INJ_GAS, RATE, 50000.0, np.array([cell_id(nx, ny, 0, 0, 0)], np.int32)),
        Well(PROD, BHP, 1000.0, np.array([cell_id(nx, ny, 9, 9, 2)], np.int32)),
    ]
    return Reservoir(
        name="c1_blackoil_10x10x3", nx=nx, ny=ny, nz=nz,
        dx=np.full(nx, 1000.0), dy=np.full(ny, 1000.0), dz=dz_l, top=8000.0,
        kx=kh.copy(), ky=kh.copy(), kz=kh / 10.0, poro=np.full(n, 0.3),
        cr=3e-6, pref=4800.0, fluid=fl, wells=wells,
        p0=np.full(n, 4800.0), sw0=np.full(n, 0.12), x0=np.full(n, rs0),
        flag0=np.full(n, UNSAT, np.int8), schedule=[30.0] * 10,
        options=Options(max_lin=300),
    )


def five_spot(nx, ny, nz, dx, dy, dz, sigma, seed, inj_rate, prod_bhp=4000.0,
              p0=5500.0, sw0=0.2, nsteps=20, dt=10.0, homogeneous_k=None,
              name="fivespot") -> Reservoir:
    """Two-phase dead-oil five-spot: central water injector over all layers at
    a surface-rate target, four corner BHP producers over all layers."""
    n = nx * ny * nz
    if homogeneous_k is not None:
        kh = np.full(n, float(homogeneous_k))
        poro = np.full(n, 0.2)
    else:
        kh, poro = lognormal_perm(nx, ny, nz, sigma, seed)
    fl = deadoil_fluid()
    ic, jc = (nx - 1) // 2, (ny - 1) // 2
    wells = [Well(INJ_WATER, RATE, float(inj_rate), column_cells(nx, ny, nz, ic, jc))]
    for (i, j) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
        wells.append(Well(PROD, BHP, prod_bhp, column_cells(nx, ny, nz, i, j)))
    return Reservoir(
        name=name, nx=nx, ny=ny, nz=nz,
        dx=np.full(nx, float(dx)), dy=np.full(ny, float(dy)), dz=np.full(nz, float(dz)),
        top=8000.0, kx=kh.copy(), ky=kh.copy(), kz=0.1 * kh, poro=poro,
        cr=3e-6, pref=p0, fluid=fl, wells=wells,
        p0=np.full(n, p0), sw0=np.full(n, sw0), x0=np.zeros(n),
        flag0=np.zeros(n, np.int8), schedule=[dt] * nsteps,
    )


def config_c2() -> Reservoir:
    """60x220x85 = 1,122,000-cell two-phase dead-oil five-spot (SPE10-shaped),
    log-normal perm sigma = 2.0, 2x2 blocks, 20 steps of 10 days."""
    return five_spot(60, 220, 85, 20.0, 10.0, 2.0, sigma=2.0, seed=20610862,
                     inj_rate=8000.0, name="c2_deadoil_60x220x85")


def config_c2_small(nx=12, ny=20, nz=6, sigma=2.0, seed=20610862, nsteps=3,
                    rate_frac=None) -> Reservoir:
    """A shrunken c2 (same cell sizes, fluid, wells and perm recipe) for parity
    cases the oracle finishes in seconds.  The injection rate is scaled by the
    cell count so the fraction of pore volume injected per step matches c2."""
    n = nx * ny * nz
    rate = 8000.0 * n / 1_122_000.0 if rate_frac is None else rate_frac
    return five_spot(nx, ny, nz, 20.0, 10.0, 2.0, sigma=sigma, seed=seed,
                     inj_rate=rate, nsteps=nsteps, name=f"c2like_{nx}x{ny}x{nz}")


def config_c3(nx=200, ny=200, nz=50) -> Reservoir:
    """Three-phase black oil on 200x200x50, sigma = 1.5, 3x3 blocks."""
    n = nx * ny * nz
    kh, poro = lognormal_perm(nx, ny, nz, 1.5, 30610862)
    fl = blackoil_fluid(swc=0.12, sor=0.10)
    rs0 = rs_sat_table(fl, 4000.0)
    dx, dy, dz = 100.0, 100.0, 5.0
    pv_rb = float(np.sum(dx * dy * dz * poro)) / 5.615
    bg_inj = float(np.interp(4800.0, fl.p, fl.bg))
    rate = 0.02 * pv_rb / bg_inj / 300.0          # Mscf/d, 2% of PV over 300 days
    ic, jc = (nx - 1) // 2, (ny - 1) // 2
    wells = [Well(INJ_GAS, RATE, rate, column_cells(nx, ny, nz, ic, jc))]
    for (i, j) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
        wells.append(Well(PROD, BHP, 1000.0, column_cells(nx, ny, nz, i, j)))
    return Reservoir(
        name=f"c3_blackoil_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
        dx=np.full(nx, dx), dy=np.full(ny, dy), dz=np.full(nz, dz), top=8000.0,
        kx=kh.copy(), ky=kh.copy(), kz=0.1 * kh, poro=poro, cr=3e-6, pref=4800.0,
        fluid=fl, wells=wells, p0=np.full(n, 4800.0), sw0=np.full(n, 0.12),
        x0=np.full(n, rs0), flag0=np.full(n, UNSAT, np.int8), schedule=[30.0] * 10,
    )


def config_c4_members(count=256, seed=40610862):
    """Grid sizes of the batched ensemble (nx, ny ~ U{20..64}, nz ~ U{5..16})."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(20, 65, size=count)
    ny = rng.integers(20, 65, size=count)
    nz = rng.integers(5, 17, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(nx, ny, nz)]


def config_c4_member(r, dims) -> Reservoir:
    nx, ny, nz = dims
    n = nx * ny * nz
    kh, poro = lognormal_perm(nx, ny, nz, 1.0, 41000000 + r)
    dx, dy, dz = 50.0, 50.0, 5.0
    fl = deadoil_fluid()
    pv_rb = float(np.sum(dx * dy * dz * poro)) / 5.615
    rate = 0.05 * pv_rb / 450.0
    wells = [Well(INJ_WATER, RATE, rate, column_cells(nx, ny, nz, 0, 0)),
             Well(PROD, BHP, 4000.0, column_cells(nx, ny, nz, nx - 1, ny - 1))]
    return Reservoir(
        name=f"c4_member{r}_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz,
        dx=np.full(nx, dx), dy=np.full(ny, dy), dz=np.full(nz, dz), top=8000.0,
        kx=kh.copy(), ky=kh.copy(), kz=0.1 * kh, poro=poro, cr=3e-6, pref=5500.0,
        fluid=fl, wells=wells, p0=np.full(n, 5500.0), sw0=np.full(n, 0.2),
        x0=np.zeros(n), flag0=np.zeros(n, np.int8), schedule=[15.0] * 30,
    )


def config_c5(nx=100, ny=100, nz=20, seed=50610862) -> Reservoir:
    n = nx * ny * nz
    res = five_spot(nx, ny, nz, 50.0, 50.0, 5.0, sigma=1.0, seed=seed,
                    inj_rate=1.0, nsteps=20, dt=30.0, name=f"c5_deadoil_{nx}x{ny}x{nz}")
    pv_rb = float(np.sum(50.0 * 50.0 * 5.0 * res.poro)) / 5.615
    res.wells[0].target = 0.10 * pv_rb / 600.0
    return res


# ----------------------------------------------------------------------------
# small analytic set-ups used by the oracle pins


def buckley_leverett_1d(ncell, length=1000.0, area=100.0, poro=0.2, rate=None,
                        t_end=None, muw=1.0, muo=1.0, swc=0.2, sor=0.2, nsteps=None):
    """1 x N x 1 incompressible two-phase displacement, no gravity.  Water is
    injected at a surface-rate target into cell 0, cell N-1 produces at
    constant BHP.  All compressibilities are zero and every FVF is 1."""
    dxy = length / ncell
    p = table_pressures()
    fl = Fluid(model=DEADOIL_OW, p=p, bo=np.ones_like(p), rs=np.zeros_like(p),
               muo=np.full_like(p, muo), bg=np.ones_like(p), mug=np.ones_like(p),
               bw_ref=1.0, cw=0.0, muw=muw, pw_ref=14.7, swc=swc, sor=sor)
    n = ncell
    pv_total = length * area * poro / 5.615   # rb
    if rate is None:
        rate = 0.1 * pv_total / 100.0              # 0.1 PV per 100 days
    if t_end is None:
        t_end = 100.0
    if nsteps is None:
        nsteps = ncell // 4
    wells = [Well(INJ_WATER, RATE, rate, np.array([0], np.int32), wi=np.array([1e4])),
             Well(PROD, BHP, 1000.0, np.array([n - 1], np.int32), wi=np.array([1e4]))]
    k = np.full(n, 1000.0)
    res = Reservoir(
        name=f"bl_{ncell}", nx=1, ny=n, nz=1, dx=np.array([np.sqrt(area)]),
        dy=np.full(n, dxy), dz=np.array([np.sqrt(area)]), top=8000.0,
        kx=k, ky=k.copy(), kz=k.copy(), poro=np.full(n, poro), cr=0.0, pref=2000.0,
        fluid=fl, wells=wells, p0=np.full(n, 2000.0), sw0=np.full(n, swc),
        x0=np.zeros(n), flag0=np.zeros(n, np.int8), schedule=[t_end / nsteps] * nsteps,
    )
    return res
