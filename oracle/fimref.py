"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Argument marshalling only; every number comes from oracle/fimref.c.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)
i8p = C.POINTER(C.c_int8)


class FrInput(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("dx", f64p), ("dy", f64p), ("dz", f64p), ("top", C.c_double),
        ("kx", f64p), ("ky", f64p), ("kz", f64p), ("poro", f64p),
        ("cr", C.c_double), ("pref", C.c_double),
        ("model", C.c_int32), ("nrows", C.c_int32),
        ("tp", f64p), ("tbo", f64p), ("trs", f64p), ("tmuo", f64p), ("tbg", f64p), ("tmug", f64p),
        ("co_us", C.c_double), ("cmu_us", C.c_double),
        ("bw_ref", C.c_double), ("cw", C.c_double), ("muw", C.c_double), ("pw_ref", C.c_double),
        ("rho_w_sc", C.c_double), ("rho_o_sc", C.c_double), ("rho_g_sc", C.c_double),
        ("swc", C.c_double), ("sor", C.c_double), ("sgc", C.c_double),
        ("nw", C.c_double), ("no", C.c_double), ("ng", C.c_double),
        ("krw_max", C.c_double), ("kro_max", C.c_double), ("krg_max", C.c_double),
        ("nwells", C.c_int32),
        ("wkind", i32p), ("wctrl", i32p),
        ("wtarget", f64p), ("wrw", f64p), ("wskin", f64p),
        ("wperf_start", i32p), ("wperf_cell", i32p), ("wperf_wi", f64p),
    ]


class FrOptions(C.Structure):
    _fields_ = [
        ("tol_cnv", C.c_double), ("tol_mb", C.c_double), ("tol_dp", C.c_double),
        ("tol_ds", C.c_double), ("tol_well", C.c_double),
        ("ds_max", C.c_double), ("dp_max", C.c_double), ("lin_rtol", C.c_double),
        ("max_newton", C.c_int32), ("max_lin", C.c_int32), ("restart", C.c_int32),
        ("max_cuts", C.c_int32), ("dense_max", C.c_int32), ("pad", C.c_int32),
        ("linsolve", C.c_void_p), ("linsolve_ctx", C.c_void_p),
    ]


# signature of FrOptions.linsolve (a ctypes callback; keep a reference to it)
LINSOLVE_FN = C.CFUNCTYPE(C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                          C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double),
                          C.POINTER(C.c_double), C.POINTER(C.c_int32))


MAX_SUB = 256


class FrReport(C.Structure):
    _fields_ = [
        ("newton_iters", C.c_int32), ("linear_iters", C.c_int32), ("cuts", C.c_int32),
        ("converged", C.c_int32), ("nsub", C.c_int32), ("pad", C.c_int32),
        ("cnv", C.c_double * 3), ("mb", C.c_double * 3),
        ("dt_sub", C.c_double * MAX_SUB),
        ("t_assemble", C.c_double), ("t_linear", C.c_double), ("t_update", C.c_double),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.fr_create.restype = C.c_void_p
        L.fr_create.argtypes = [C.POINTER(FrInput)]
        L.fr_destroy.argtypes = [C.c_void_p]
        L.fr_error.restype = C.c_char_p
        for f in ("fr_ncells", "fr_nb", "fr_nwells", "fr_nperf", "fr_nnzb", "fr_nprops"):
            getattr(L, f).restype = C.c_int32
            getattr(L, f).argtypes = [C.c_void_p]
        L.fr_static.argtypes = [C.c_void_p] + [f64p] * 7
        L.fr_pattern.argtypes = [C.c_void_p, i32p, i32p]
        L.fr_props.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p]
        L.fr_accum.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p]
        L.fr_assemble.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p, f64p, C.c_double,
                                  f64p, f64p]
        L.fr_well_rates.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p, f64p]
        L.fr_conv.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p, C.c_double, f64p, f64p]
        L.fr_bsr_spmv.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p, f64p]
        L.fr_bj_setup.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p]
        L.fr_bj_apply.argtypes = [C.c_int32, C.c_int32, f64p, f64p, f64p]
        L.fr_bilu0_factor.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p]
        L.fr_bilu0_solve.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p, f64p]
        L.fr_dense_solve.argtypes = [C.c_int32, f64p, f64p]
        L.fr_gmres_bilu0.argtypes = [C.c_int32, C.c_int32, i32p, i32p, f64p, f64p, f64p,
                                     C.c_double, C.c_int32, C.c_int32, i32p, f64p]
        L.fr_step.argtypes = [C.c_void_p, f64p, f64p, f64p, i8p, f64p, C.c_double,
                              C.POINTER(FrOptions), C.POINTER(FrReport)]
        _LIB = L
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleModel:
    """One reservoir loaded into the oracle, with its own state copy."""

    def __init__(self, res):
        L = lib()
        self.res = res
        fl = res.fluid
        keep = []

        def d(a):
            a = _f64(a)
            keep.append(a)
            return _p(a, f64p)

        def i(a):
            a = np.ascontiguousarray(a, dtype=np.int32)
            keep.append(a)
            return _p(a, i32p)

        wells = res.wells
        starts = np.zeros(len(wells) + 1, np.int32)
        cells, wis = [], []
        for k, w in enumerate(wells):
            starts[k + 1] = starts[k] + len(w.cells)
            cells.append(np.asarray(w.cells, np.int32))
            wis.append(np.asarray(w.wi, np.float64) if w.wi is not None
                       else np.zeros(len(w.cells)))
        cells = np.concatenate(cells) if cells else np.zeros(0, np.int32)
        wis = np.concatenate(wis) if wis else np.zeros(0)
        inp = FrInput(
            nx=res.nx, ny=res.ny, nz=res.nz, dx=d(res.dx), dy=d(res.dy), dz=d(res.dz),
            top=res.top, kx=d(res.kx), ky=d(res.ky), kz=d(res.kz), poro=d(res.poro),
            cr=res.cr, pref=res.pref, model=fl.model, nrows=len(fl.p),
            tp=d(fl.p), tbo=d(fl.bo), trs=d(fl.rs), tmuo=d(fl.muo), tbg=d(fl.bg), tmug=d(fl.mug),
            co_us=fl.co_us, cmu_us=fl.cmu_us, bw_ref=fl.bw_ref, cw=fl.cw, muw=fl.muw,
            pw_ref=fl.pw_ref, rho_w_sc=fl.rho_sc[0], rho_o_sc=fl.rho_sc[1], rho_g_sc=fl.rho_sc[2],
            swc=fl.swc, sor=fl.sor, sgc=fl.sgc, nw=fl.nw, no=fl.no, ng=fl.ng,
            krw_max=fl.krw_max, kro_max=fl.kro_max, krg_max=fl.krg_max,
            nwells=len(wells),
            wkind=i([w.kind for w in wells] or [0]), wctrl=i([w.control for w in wells] or [0]),
            wtarget=d([w.target for w in wells] or [0.0]), wrw=d([w.rw for w in wells] or [0.0]),
            wskin=d([w.skin for w in wells] or [0.0]),
            wperf_start=i(starts), wperf_cell=i(cells if len(cells) else [0]),
            wperf_wi=d(wis if len(wis) else [0.0]),
        )
        h = L.fr_create(C.byref(inp))
        if not h:
            raise ValueError("oracle rejected input: " + L.fr_error().decode())
        self.h = C.c_void_p(h)
        self.n = L.fr_ncells(self.h)
        self.nb = L.fr_nb(self.h)
        self.nw = L.fr_nwells(self.h)
        self.nperf = L.fr_nperf(self.h)
        self.nnzb = L.fr_nnzb(self.h)
        self.nprops = L.fr_nprops(self.h)
        self.nrows = self.n + self.nw
        # state
        self.P = _f64(res.p0).copy()
        self.Sw = _f64(res.sw0).copy()
        self.X = _f64(res.x0).copy()
        self.flag = np.ascontiguousarray(res.flag0, dtype=np.int8).copy()
        self.pbhp = np.array([self.initial_bhp(w) for w in wells], dtype=np.float64)

    def initial_bhp(self, w):
        if w.bhp0 is not None:
            return float(w.bhp0)
        if w.control == 0:
            return float(w.target)
        return float(np.mean(np.asarray(self.res.p0)[np.asarray(w.cells)]))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().fr_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- static / pattern ----------------------------------------------------
    def static(self):
        n = self.n
        out = [np.zeros(n) for _ in range(6)] + [np.zeros(max(self.nperf, 1))]
        lib().fr_static(self.h, *[_p(a, f64p) for a in out])
        keys = ["vol", "depth", "pvref", "tx", "ty", "tz", "wi"]
        res = dict(zip(keys, out))
        res["wi"] = res["wi"][: self.nperf]
        return res

    def pattern(self):
        rowptr = np.zeros(self.nrows + 1, np.int32)
        colind = np.zeros(self.nnzb, np.int32)
        lib().fr_pattern(self.h, _p(rowptr, i32p), _p(colind, i32p))
        return rowptr, colind

    # -- state-dependent evaluations --------------------------------------------
    def _st(self, P=None, Sw=None, X=None, flag=None, pbhp=None):
        P = _f64(self.P if P is None else P)
        Sw = _f64(self.Sw if Sw is None else Sw)
        X = _f64(self.X if X is None else X)
        flag = np.ascontiguousarray(self.flag if flag is None else flag, dtype=np.int8)
        pbhp = _f64(self.pbhp if pbhp is None else pbhp)
        if pbhp.size == 0:
            pbhp = np.zeros(1)
        return P, Sw, X, flag, pbhp

    def props(self, **st):
        P, Sw, X, flag, _ = self._st(**st)
        out = np.zeros(self.nprops * self.n)
        lib().fr_props(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p), _p(flag, i8p),
                       _p(out, f64p))
        return out.reshape(self.nprops, self.n)

    def accum(self, **st):
        P, Sw, X, flag, _ = self._st(**st)
        A = np.zeros(self.n * self.nb)
        lib().fr_accum(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p), _p(flag, i8p),
                       _p(A, f64p))
        return A

    def assemble(self, dt, Aold=None, jacobian=True, **st):
        P, Sw, X, flag, pbhp = self._st(**st)
        if Aold is None:
            Aold = self.accum()
        Aold = _f64(Aold)
        R = np.zeros(self.nrows * self.nb)
        val = np.zeros(self.nnzb * self.nb * self.nb) if jacobian else None
        lib().fr_assemble(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p), _p(flag, i8p),
                          _p(pbhp, f64p), _p(Aold, f64p), float(dt), _p(R, f64p),
                          _p(val, f64p) if val is not None else None)
        return R, val

    def well_rates(self, **st):
        P, Sw, X, flag, pbhp = self._st(**st)
        q = np.zeros(max(self.nw, 1) * 3)
        lib().fr_well_rates(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p), _p(flag, i8p),
                            _p(pbhp, f64p), _p(q, f64p))
        return q[: self.nw * 3].reshape(self.nw, 3)

    def conv(self, R, dt, **st):
        P, Sw, X, flag, _ = self._st(**st)
        cnv = np.zeros(3)
        mb = np.zeros(3)
        R = _f64(R)
        lib().fr_conv(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p), _p(flag, i8p),
                      _p(R, f64p), float(dt), _p(cnv, f64p), _p(mb, f64p))
        return cnv, mb

    # -- stepping -----------------------------------------------------------------
    def options(self, dense_max=1200, **over):
        o = self.res.options
        opt = FrOptions(tol_cnv=o.tol_cnv, tol_mb=o.tol_mb, tol_dp=o.tol_dp, tol_ds=o.tol_ds,
                        tol_well=o.tol_well, ds_max=o.ds_max, dp_max=o.dp_max,
                        lin_rtol=min(o.lin_rtol, 1e-12), max_newton=o.max_newton,
                        max_lin=max(o.max_lin, 2000), restart=50, max_cuts=o.max_cuts,
                        dense_max=dense_max)
        for k, v in over.items():
            setattr(opt, k, v)
        return opt

    def step(self, dt, opt=None):
        if opt is None:
            opt = self.options()
        rep = FrReport()
        pb = self.pbhp if self.pbhp.size else np.zeros(1)
        st = lib().fr_step(self.h, _p(self.P, f64p), _p(self.Sw, f64p), _p(self.X, f64p),
                           _p(self.flag, i8p), _p(pb, f64p), float(dt), C.byref(opt),
                           C.byref(rep))
        if self.pbhp.size:
            self.pbhp[:] = pb[: self.nw]
        return st, rep

    def state(self):
        return dict(P=self.P.copy(), Sw=self.Sw.copy(), X=self.X.copy(),
                    flag=self.flag.copy(), pbhp=self.pbhp.copy())

    def set_state(self, P, Sw, X, flag, pbhp=None):
        self.P[:] = P
        self.Sw[:] = Sw
        self.X[:] = X
        self.flag[:] = flag
        if pbhp is not None:
            self.pbhp[:] = pbhp


# -- free-standing linear algebra --------------------------------------------------

def bsr_spmv(rowptr, colind, val, x, nb):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    colind = np.ascontiguousarray(colind, np.int32)
    val = _f64(val)
    x = _f64(x)
    nrows = len(rowptr) - 1
    y = np.zeros(nrows * nb)
    lib().fr_bsr_spmv(nrows, nb, _p(rowptr, i32p), _p(colind, i32p), _p(val, f64p),
                      _p(x, f64p), _p(y, f64p))
    return y


def bj_setup(rowptr, colind, val, nb):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    colind = np.ascontiguousarray(colind, np.int32)
    val = _f64(val)
    nrows = len(rowptr) - 1
    dinv = np.zeros(nrows * nb * nb)
    st = lib().fr_bj_setup(nrows, nb, _p(rowptr, i32p), _p(colind, i32p), _p(val, f64p),
                           _p(dinv, f64p))
    if st:
        raise ValueError("singular diagonal block")
    return dinv


def bj_apply(dinv, x, nb):
    dinv = _f64(dinv)
    x = _f64(x)
    nrows = x.size // nb
    y = np.zeros_like(x)
    lib().fr_bj_apply(nrows, nb, _p(dinv, f64p), _p(x, f64p), _p(y, f64p))
    return y


def bilu0(rowptr, colind, val, nb):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    colind = np.ascontiguousarray(colind, np.int32)
    val = _f64(val)
    lu = np.zeros_like(val)
    st = lib().fr_bilu0_factor(len(rowptr) - 1, nb, _p(rowptr, i32p), _p(colind, i32p),
                               _p(val, f64p), _p(lu, f64p))
    if st:
        raise ValueError("singular pivot block")
    return lu


def bilu0_solve(rowptr, colind, lu, b, nb):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    colind = np.ascontiguousarray(colind, np.int32)
    lu = _f64(lu)
    b = _f64(b)
    x = np.zeros_like(b)
    lib().fr_bilu0_solve(len(rowptr) - 1, nb, _p(rowptr, i32p), _p(colind, i32p), _p(lu, f64p),
                         _p(b, f64p), _p(x, f64p))
    return x


def ilu_tiles(nx, ny, nz, tile, well_cells):
    """Subdomains of block-Jacobi ILU(0) (Sec. 5.1: block Jacobi over
    subdomains with ILU(0) inside each).  Cell (i, j, k) belongs to the box
    (i // tx, j // ty, k // tz); a well row joins the box that holds all of
    its perforated cells, otherwise it is a subdomain of its own.  Returns the
    subdomain id of every row (cells, then wells)."""
    tx, ty, tz = tile
    ntx, nty = -(-nx // tx), -(-ny // ty)
    c = np.arange(nx * ny * nz)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    cell_tile = (i // tx) + ntx * ((j // ty) + nty * (k // tz))
    nt = int(cell_tile.max()) + 1 if len(c) else 0
    wt = []
    for w, cells in enumerate(well_cells):
        ts = set(int(cell_tile[q]) for q in cells)
        wt.append(ts.pop() if len(ts) == 1 else nt + w)
    return np.concatenate([cell_tile, np.array(wt, dtype=np.int64)])


def bilu0_tiled(rowptr, colind, val, nb, row_tile):
    """ILU(0) inside each subdomain: the natural-order BILU(0) of A with every
    block that couples two different subdomains set to zero.  A zero coupling
    adds nothing to any update, so the factors of each subdomain are those of
    its own diagonal part and every cross-subdomain block stays zero."""
    rowptr = np.asarray(rowptr)
    colind = np.asarray(colind)
    rows = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    keep = row_tile[rows] == row_tile[colind]
    v = _f64(val).reshape(-1, nb * nb).copy()
    v[~keep] = 0.0
    return bilu0(rowptr, colind, v.reshape(-1), nb)


def dense_solve(A, b):
    A = np.array(A, dtype=np.float64, order="C")
    b = np.array(b, dtype=np.float64)
    st = lib().fr_dense_solve(len(b), _p(A, f64p), _p(b, f64p))
    if st:
        raise ValueError("singular matrix")
    return b


def gmres_bilu0(rowptr, colind, val, b, nb, rtol=1e-12, restart=50, max_iter=2000):
    rowptr = np.ascontiguousarray(rowptr, np.int32)
    colind = np.ascontiguousarray(colind, np.int32)
    val = _f64(val)
    b = _f64(b)
    x = np.zeros_like(b)
    it = C.c_int32(0)
    rr = C.c_double(0)
    st = lib().fr_gmres_bilu0(len(rowptr) - 1, nb, _p(rowptr, i32p), _p(colind, i32p),
                              _p(val, f64p), _p(b, f64p), _p(x, f64p), rtol, restart, max_iter,
                              C.byref(it), C.byref(rr))
    return x, st, it.value, rr.value


def bsr_to_dense(rowptr, colind, val, nb):
    nrows = len(rowptr) - 1
    A = np.zeros((nrows * nb, nrows * nb))
    v = np.asarray(val).reshape(-1, nb, nb)
    for r in range(nrows):
        for q in range(rowptr[r], rowptr[r + 1]):
            c = colind[q]
            A[r * nb:(r + 1) * nb, c * nb:(c + 1) * nb] = v[q]
    return A


def prop_index(nb):
    """Names of the rows of the property record (same order as fimref.h)."""
    names = []
    phases = ["w", "o", "g"][:nb]
    unk = ["P", "Sw", "X"][:nb]

    def group(base):
        names.append(base)
        for u in unk:
            names.append(f"d{base}_d{u}")

    for j in phases:
        group(f"Lam_{j}")
    if nb == 3:
        group("Lam_og")
    group("lam_t")
    for j in phases:
        group(f"gam_{j}")
    for i in phases:
        group(f"A_{i}")
    for j in phases:
        names.append(f"b_{j}")
    names.append("PV")
    return {n: k for k, n in enumerate(names)}
