"""ctypes binding of libfim.so (include/fim.h).  Argument marshalling only:
every numeric step runs in the library's HIP kernels.

The library must have been built (``python -m paper_2406_10862_amd.build``
or ``__graft_entry__.build()``); importing this module never falls back to
anything else, it raises when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import reservoirs as rv

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfim.so")

FIM_OK, FIM_NOT_CONVERGED, FIM_SKIPPED = 0, 1, 2
FIM_E_ARG, FIM_E_NOMEM, FIM_E_HIP, FIM_E_STATE = -1, -2, -3, -4
FIM_MAX_SUB = 256

i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)
i8p = C.POINTER(C.c_int8)


class FimGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", f64p), ("dy", f64p), ("dz", f64p), ("top", C.c_double)]


class FimRock(C.Structure):
    _fields_ = [("kx", f64p), ("ky", f64p), ("kz", f64p), ("poro", f64p),
                ("cr", C.c_double), ("pref", C.c_double)]


class FimFluid(C.Structure):
    _fields_ = [("model", C.c_int32), ("nrows", C.c_int32),
                ("p", f64p), ("bo", f64p), ("rs", f64p), ("muo", f64p), ("bg", f64p),
                ("mug", f64p), ("co_us", C.c_double), ("cmu_us", C.c_double),
                ("bw_ref", C.c_double), ("cw", C.c_double), ("muw", C.c_double),
                ("pw_ref", C.c_double), ("rho_sc", C.c_double * 3),
                ("swc", C.c_double), ("sor", C.c_double), ("sgc", C.c_double),
                ("nw", C.c_double), ("no", C.c_double), ("ng", C.c_double),
                ("krw_max", C.c_double), ("kro_max", C.c_double), ("krg_max", C.c_double)]


class FimWell(C.Structure):
    _fields_ = [("kind", C.c_int32), ("control", C.c_int32), ("target", C.c_double),
                ("nperf", C.c_int32), ("cells", i32p), ("wi", f64p),
                ("rw", C.c_double), ("skin", C.c_double)]


class FimOptions(C.Structure):
    _fields_ = [("tol_cnv", C.c_double), ("tol_mb", C.c_double), ("tol_dp", C.c_double),
                ("tol_ds", C.c_double), ("tol_well", C.c_double), ("ds_max", C.c_double),
                ("dp_max", C.c_double), ("lin_rtol", C.c_double),
                ("max_newton", C.c_int32), ("max_lin", C.c_int32), ("restart", C.c_int32),
                ("max_cuts", C.c_int32), ("precond", C.c_int32), ("precision", C.c_int32),
                ("profile", C.c_int32), ("amg_cycle", C.c_int32), ("amg_sweeps", C.c_int32),
                ("graphs", C.c_int32), ("forcing", C.c_int32), ("amg_fused", C.c_int32),
                ("tile_nx", C.c_int32), ("tile_ny", C.c_int32), ("tile_nz", C.c_int32),
                ("amg_seg_rows", C.c_int32), ("gs_refine", C.c_int32), ("amg_exact", C.c_int32),
                ("amg_exact_mode", C.c_int32)]


class FimStepReport(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("linear_iters", C.c_int32),
                ("cuts", C.c_int32), ("converged", C.c_int32), ("nsub", C.c_int32),
                ("spmv_calls", C.c_int32), ("dt_done", C.c_double),
                ("cnv", C.c_double * 3), ("mb", C.c_double * 3),
                ("t_assemble", C.c_double), ("t_linear", C.c_double),
                ("t_update", C.c_double), ("spmv_ms", C.c_double),
                ("last_dp", C.c_double), ("last_ds", C.c_double), ("well_res", C.c_double),
                ("dt_sub", C.c_double * FIM_MAX_SUB), ("gs_vectors", C.c_double)]


class FimAdjointReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("substeps", C.c_int32), ("cuts", C.c_int32),
                ("newton_iters", C.c_int32), ("linear_iters", C.c_int32),
                ("adjoint_iters", C.c_int32), ("objective", C.c_double),
                ("adjoint_relres", C.c_double), ("t_forward_ms", C.c_double),
                ("t_adjoint_ms", C.c_double), ("t_recompute_ms", C.c_double),
                ("stored_states", C.c_int32), ("pad", C.c_int32)]


class FimTuneReport(C.Structure):
    _fields_ = [("box", C.c_int32 * 3), ("from_cache", C.c_int32), ("trials", C.c_int32),
                ("ncand", C.c_int32), ("cand", (C.c_int32 * 3) * 16),
                ("trial_ms", C.c_double * 16)]


EXPORTS = ["fim_create", "fim_destroy", "fim_last_error", "fim_sizes", "fim_set_options",
           "fim_set_state", "fim_set_state_dev", "fim_get_state", "fim_step",
           "fim_get_well_rates", "fim_static", "fim_set_iterate", "fim_props",
           "fim_assemble", "fim_precond_apply", "fim_linear_solve", "fim_bsr_spmv",
           "fim_ensemble_run", "fim_adjoint_gradient", "fim_step_noalloc", "fim_set_perm",
           "fim_set_perm_dev", "fim_ensemble_tune", "fim_amg_level", "fim_amg_coarse_solve"]

_LIB = None


class FimError(RuntimeError):
    pass


def lib():
    """Load libfim.so; raises when it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise FimError(f"{LIB_PATH} is missing: build it with "
                       "`python -m paper_2406_10862_amd.build` (no fallback path exists)")
    # torch bundles its own HIP runtime under the same soname as the system
    # one; it must be the first one loaded so that the library binds to the
    # runtime that owns the device and the streams torch hands out
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.fim_create.argtypes = [C.POINTER(FimGrid), C.POINTER(FimRock), C.POINTER(FimFluid),
                             C.c_int32, C.POINTER(FimWell), C.POINTER(FimOptions), vp,
                             C.POINTER(vp)]
    L.fim_destroy.argtypes = [vp]
    L.fim_destroy.restype = None
    L.fim_last_error.restype = C.c_char_p
    L.fim_sizes.argtypes = [vp, i32p, i32p, i32p, i32p, i32p]
    L.fim_set_options.argtypes = [vp, C.POINTER(FimOptions)]
    for f in ("fim_set_state", "fim_set_iterate"):
        getattr(L, f).argtypes = [vp, f64p, f64p, f64p, i8p, f64p]
    L.fim_set_state_dev.argtypes = [vp, vp, vp, vp, vp, f64p]
    L.fim_get_state.argtypes = [vp, f64p, f64p, f64p, i8p, f64p]
    L.fim_step.argtypes = [vp, C.c_double, C.POINTER(FimStepReport)]
    L.fim_step_noalloc.argtypes = [vp, C.c_double, C.POINTER(FimStepReport)]
    L.fim_get_well_rates.argtypes = [vp, f64p, f64p]
    L.fim_static.argtypes = [vp] + [f64p] * 7
    L.fim_props.argtypes = [vp, f64p]
    L.fim_assemble.argtypes = [vp, C.c_double, f64p, i32p, i32p, f64p]
    L.fim_precond_apply.argtypes = [vp, f64p, f64p]
    L.fim_linear_solve.argtypes = [vp, f64p, f64p, i32p, f64p]
    L.fim_bsr_spmv.argtypes = [C.c_int32, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.fim_adjoint_gradient.argtypes = [vp, C.c_int32, f64p, f64p, C.c_int32, f64p,
                                       C.POINTER(FimAdjointReport)]
    L.fim_set_perm.argtypes = [vp, f64p, f64p, f64p]
    L.fim_amg_level.argtypes = [vp, C.c_int32, i32p, f64p]
    L.fim_amg_coarse_solve.argtypes = [vp, f64p, f64p]
    L.fim_ensemble_tune.argtypes = [C.c_int32, C.POINTER(vp), C.c_double, C.c_int32, C.c_char_p,
                                    C.POINTER(FimTuneReport)]
    L.fim_set_perm_dev.argtypes = [vp, vp, vp, vp]
    L.fim_ensemble_run.argtypes = [C.c_int32, C.POINTER(vp), C.c_int32, f64p,
                                   C.POINTER(FimStepReport), i32p]
    for f in EXPORTS:
        if f not in ("fim_destroy", "fim_last_error"):
            getattr(L, f).restype = C.c_int32
    _LIB = L
    return L


def _check(rc, what):
    if rc < 0:
        raise FimError(f"{what} failed ({rc}): {lib().fim_last_error().decode()}")
    return rc


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _tensor_shape(t, dtype, numel, name):
    import torch

    if not isinstance(t, torch.Tensor):
        raise FimError(f"{name}: a torch tensor is required, got {type(t).__name__}")
    if t.dtype != dtype:
        raise FimError(f"{name}: dtype {t.dtype}, {dtype} required")
    if not t.is_contiguous():
        raise FimError(f"{name}: the tensor must be contiguous")
    if t.numel() != numel:
        raise FimError(f"{name}: {t.numel()} elements, {numel} required")


def _tensor_device(t, name, device):
    if t.device.type != "cuda":
        raise FimError(f"{name}: a GPU tensor is required, got device {t.device}")
    if device is not None and t.device.index != device:
        raise FimError(f"{name}: on cuda:{t.device.index}, the context is on cuda:{device}")


def dev_ptr(t, dtype, numel, name, device=None):
    """data_ptr() of a torch tensor handed to a "_dev" entry point, after
    checking what the library takes on trust: element type, contiguity,
    element count and a GPU device (the given one when set).  Raises FimError
    before anything is launched."""
    _tensor_shape(t, dtype, numel, name)
    _tensor_device(t, name, device)
    return C.c_void_p(t.data_ptr())


def current_stream():
    """hipStream_t of torch's current stream, or NULL without torch/GPU."""
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(0)


def _current_device():
    """torch's current GPU index, or None without a GPU."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_device()
    except Exception:
        pass
    return None


def options_struct(o: rv.Options, profile=False) -> FimOptions:
    return FimOptions(tol_cnv=o.tol_cnv, tol_mb=o.tol_mb, tol_dp=o.tol_dp, tol_ds=o.tol_ds,
                      tol_well=o.tol_well, ds_max=o.ds_max, dp_max=o.dp_max,
                      lin_rtol=o.lin_rtol, max_newton=o.max_newton, max_lin=o.max_lin,
                      restart=o.restart, max_cuts=o.max_cuts, precond=o.precond,
                      precision=o.precision, profile=int(profile),
                      amg_cycle=o.amg_cycle, amg_sweeps=o.amg_sweeps, graphs=o.graphs,
                      forcing=o.forcing, amg_fused=o.amg_fused,
                      tile_nx=o.tile[0], tile_ny=o.tile[1], tile_nz=o.tile[2],
                      amg_seg_rows=o.amg_seg_rows, gs_refine=o.gs_refine,
                      amg_exact=o.amg_exact, amg_exact_mode=o.amg_exact_mode)


class Fim:
    """One fim_ctx built from a seeded reservoir description."""

    def __init__(self, res: rv.Reservoir, options: rv.Options | None = None, stream=None,
                 profile=False):
        L = lib()
        self.res = res
        fl = res.fluid
        self._keep = []

        def d(a):
            a = _f64(a)
            self._keep.append(a)
            return _p(a, f64p)

        grid = FimGrid(res.nx, res.ny, res.nz, d(res.dx), d(res.dy), d(res.dz), res.top)
        rock = FimRock(d(res.kx), d(res.ky), d(res.kz), d(res.poro), res.cr, res.pref)
        fluid = FimFluid(model=fl.model, nrows=len(fl.p), p=d(fl.p), bo=d(fl.bo), rs=d(fl.rs),
                         muo=d(fl.muo), bg=d(fl.bg), mug=d(fl.mug), co_us=fl.co_us,
                         cmu_us=fl.cmu_us, bw_ref=fl.bw_ref, cw=fl.cw, muw=fl.muw,
                         pw_ref=fl.pw_ref, rho_sc=(C.c_double * 3)(*fl.rho_sc), swc=fl.swc,
                         sor=fl.sor, sgc=fl.sgc, nw=fl.nw, no=fl.no, ng=fl.ng,
                         krw_max=fl.krw_max, kro_max=fl.kro_max, krg_max=fl.krg_max)
        wells = (FimWell * max(len(res.wells), 1))()
        for k, w in enumerate(res.wells):
            cells = np.ascontiguousarray(w.cells, dtype=np.int32)
            self._keep.append(cells)
            wi = d(w.wi) if w.wi is not None else None
            wells[k] = FimWell(kind=w.kind, control=w.control, target=w.target,
                               nperf=len(cells), cells=_p(cells, i32p), wi=wi, rw=w.rw,
                               skin=w.skin)
        self.options = options if options is not None else res.options
        opt = options_struct(self.options, profile)
        self.stream = current_stream() if stream is None else stream
        self.device = _current_device()
        h = C.c_void_p()
        _check(L.fim_create(C.byref(grid), C.byref(rock), C.byref(fluid), len(res.wells),
                            wells, C.byref(opt), self.stream, C.byref(h)), "fim_create")
        self.h = h
        n, nb, nw, nnzb, npr = (C.c_int32() for _ in range(5))
        _check(L.fim_sizes(self.h, C.byref(n), C.byref(nb), C.byref(nw), C.byref(nnzb),
                           C.byref(npr)), "fim_sizes")
        self.n, self.nb, self.nw, self.nnzb, self.nprops = (n.value, nb.value, nw.value,
                                                            nnzb.value, npr.value)
        self.nrows = self.n + self.nw
        self._keep_static = []

    def close(self):
        if getattr(self, "h", None):
            lib().fim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- options / state ---------------------------------------------------------
    def fim_set_options(self, options: rv.Options, profile=False):
        self.options = options
        _check(lib().fim_set_options(self.h, C.byref(options_struct(options, profile))),
               "fim_set_options")

    def fim_set_state(self, P, Sw, X=None, flag=None, bhp=None):
        P, Sw = _f64(P), _f64(Sw)
        X = _f64(X) if X is not None else None
        flag = np.ascontiguousarray(flag, np.int8) if flag is not None else None
        bhp = _f64(bhp) if bhp is not None and len(bhp) else None
        _check(lib().fim_set_state(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p),
                                   _p(flag, i8p), _p(bhp, f64p)), "fim_set_state")

    def fim_set_state_dev(self, P, Sw, X=None, flag=None, bhp=None):
        """Contiguous torch GPU tensors on the context's device: P, Sw, X
        float64 and flag int8, ncells elements each (X and flag may be None);
        read in order after the work on the context's stream."""
        import torch

        n, dv = self.n, self.device
        pP = dev_ptr(P, torch.float64, n, "P", dv)
        pS = dev_ptr(Sw, torch.float64, n, "Sw", dv)
        pX = dev_ptr(X, torch.float64, n, "X", dv) if X is not None else C.c_void_p(0)
        pF = dev_ptr(flag, torch.int8, n, "flag", dv) if flag is not None else C.c_void_p(0)
        bhp = _f64(bhp) if bhp is not None and len(bhp) else None
        if bhp is not None and bhp.size != self.nw:
            raise FimError(f"bhp: {bhp.size} values, {self.nw} wells")
        _check(lib().fim_set_state_dev(self.h, pP, pS, pX, pF, _p(bhp, f64p)),
               "fim_set_state_dev")

    def fim_set_iterate(self, P, Sw, X=None, flag=None, bhp=None):
        P, Sw = _f64(P), _f64(Sw)
        X = _f64(X) if X is not None else None
        flag = np.ascontiguousarray(flag, np.int8) if flag is not None else None
        bhp = _f64(bhp) if bhp is not None and len(bhp) else None
        _check(lib().fim_set_iterate(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p),
                                     _p(flag, i8p), _p(bhp, f64p)), "fim_set_iterate")

    def set_initial_state(self):
        r = self.res
        bhp = None
        self.fim_set_state(r.p0, r.sw0, r.x0, r.flag0, bhp)

    def fim_get_state(self):
        n = self.n
        P, Sw, X = np.zeros(n), np.zeros(n), np.zeros(n)
        flag = np.zeros(n, np.int8)
        bhp = np.zeros(max(self.nw, 1))
        _check(lib().fim_get_state(self.h, _p(P, f64p), _p(Sw, f64p), _p(X, f64p),
                                   _p(flag, i8p), _p(bhp, f64p)), "fim_get_state")
        return dict(P=P, Sw=Sw, X=X, flag=flag, pbhp=bhp[: self.nw])

    def fim_adjoint_gradient(self, dt, q_obs, checkpoint_every=0):
        """dJ/d(ln k) of every cell for J = sum_s sum_producers (q_o - q_obs[s, w])^2
        over the steps dt (fim_adjoint_gradient); checkpoint_every = k >= 1
        recomputes segments of k steps from checkpoints, 0 keeps every
        sub-step state.  Returns (rc, grad, report)."""
        dt = _f64(np.atleast_1d(dt))
        qo = _f64(np.asarray(q_obs, dtype=np.float64).reshape(len(dt), self.nw)) if self.nw else None
        grad = np.zeros(self.n)
        rep = FimAdjointReport()
        rc = _check(lib().fim_adjoint_gradient(self.h, len(dt), _p(dt, f64p), _p(qo, f64p),
                                               int(checkpoint_every), _p(grad, f64p),
                                               C.byref(rep)),
                    "fim_adjoint_gradient")
        return rc, grad, rep

    def fim_set_perm(self, kx, ky, kz):
        kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
        for name, a in (("kx", kx), ("ky", ky), ("kz", kz)):
            if a.size != self.n:
                raise FimError(f"{name}: {a.size} values, {self.n} cells")
        _check(lib().fim_set_perm(self.h, _p(kx, f64p), _p(ky, f64p), _p(kz, f64p)),
               "fim_set_perm")

    def fim_set_perm_dev(self, kx, ky, kz):
        """Contiguous float64 torch GPU tensors of ncells permeabilities (mD)."""
        import torch

        ptr = [dev_ptr(t, torch.float64, self.n, name, self.device)
               for t, name in ((kx, "kx"), (ky, "ky"), (kz, "kz"))]
        _check(lib().fim_set_perm_dev(self.h, *ptr), "fim_set_perm_dev")

    def fim_step(self, dt):
        rep = FimStepReport()
        rc = _check(lib().fim_step(self.h, float(dt), C.byref(rep)), "fim_step")
        return rc, rep

    def fim_step_noalloc(self, dt):
        """fim_step without device allocation (static reduction scratch,
        eager launches)."""
        rep = FimStepReport()
        rc = _check(lib().fim_step_noalloc(self.h, float(dt), C.byref(rep)), "fim_step_noalloc")
        return rc, rep

    def fim_get_well_rates(self):
        q = np.zeros(max(self.nw, 1) * 3)
        bhp = np.zeros(max(self.nw, 1))
        _check(lib().fim_get_well_rates(self.h, _p(q, f64p), _p(bhp, f64p)),
               "fim_get_well_rates")
        return q[: self.nw * 3].reshape(self.nw, 3), bhp[: self.nw]

    # -- testing hooks ---------------------------------------------------------------
    def fim_static(self):
        n = self.n
        out = [np.zeros(n) for _ in range(6)]
        nperf = sum(len(w.cells) for w in self.res.wells)
        wi = np.zeros(max(nperf, 1))
        _check(lib().fim_static(self.h, *[_p(a, f64p) for a in out], _p(wi, f64p)),
               "fim_static")
        keys = ["vol", "depth", "pvref", "tx", "ty", "tz"]
        d = dict(zip(keys, out))
        d["wi"] = wi[:nperf]
        return d

    def fim_props(self):
        out = np.zeros(self.nprops * self.n)
        _check(lib().fim_props(self.h, _p(out, f64p)), "fim_props")
        return out.reshape(self.nprops, self.n)

    def fim_assemble(self, dt, jacobian=True):
        R = np.zeros(self.nrows * self.nb)
        rowptr = np.zeros(self.nrows + 1, np.int32)
        colind = np.zeros(self.nnzb, np.int32)
        val = np.zeros(self.nnzb * self.nb * self.nb) if jacobian else None
        _check(lib().fim_assemble(self.h, float(dt), _p(R, f64p), _p(rowptr, i32p),
                                  _p(colind, i32p), _p(val, f64p)), "fim_assemble")
        return R, rowptr, colind, val

    def fim_amg_level(self, level):
        """Dense pressure operator of one AMG level of the CPR stage (cells in
        natural order, then wells) and its dims (nx, ny, nz, nwells)."""
        dims = np.zeros(4, np.int32)
        _check(lib().fim_amg_level(self.h, int(level), _p(dims, i32p), None), "fim_amg_level")
        N = int(dims[0] * dims[1] * dims[2] + dims[3])
        A = np.zeros((N, N))
        _check(lib().fim_amg_level(self.h, int(level), _p(dims, i32p), _p(A, f64p)),
               "fim_amg_level")
        return A, tuple(int(v) for v in dims)

    def fim_amg_coarse_solve(self, b):
        """The coarsest level's solve of the cycle for b (fim_amg_level order)."""
        b = _f64(b)
        x = np.zeros_like(b)
        _check(lib().fim_amg_coarse_solve(self.h, _p(b, f64p), _p(x, f64p)), "fim_amg_coarse_solve")
        return x

    def fim_amg_levels(self):
        """Number of AMG levels of the CPR stage."""
        dims = np.zeros(4, np.int32)
        n = 0
        while lib().fim_amg_level(self.h, n, _p(dims, i32p), None) == FIM_OK:
            n += 1
        return n

    def fim_precond_apply(self, x):
        x = _f64(x)
        y = np.zeros_like(x)
        _check(lib().fim_precond_apply(self.h, _p(x, f64p), _p(y, f64p)), "fim_precond_apply")
        return y

    def fim_linear_solve(self, b):
        b = _f64(b)
        x = np.zeros_like(b)
        it = C.c_int32(0)
        rr = C.c_double(0)
        rc = _check(lib().fim_linear_solve(self.h, _p(b, f64p), _p(x, f64p), C.byref(it),
                                           C.byref(rr)), "fim_linear_solve")
        return x, rc, it.value, rr.value


def fim_bsr_spmv(nrows, nb, rowptr, colind, val, x, y, stream=None):
    """y = A x on contiguous torch GPU tensors of one device (canonical BSR:
    rowptr int32 [nrows+1], colind int32 [nnzb], val float64 [nnzb*nb*nb];
    x, y float64 [nrows*nb] interleaved).  Column indices are not checked."""
    import torch

    nrows, nb = int(nrows), int(nb)
    if nb not in (2, 3) or nrows < 0:
        raise FimError(f"fim_bsr_spmv: nb {nb} (2 or 3) and nrows {nrows} (>= 0)")
    nnzb = colind.numel() if isinstance(colind, torch.Tensor) else -1
    ops = [(rowptr, torch.int32, nrows + 1, "rowptr"), (colind, torch.int32, nnzb, "colind"),
           (val, torch.float64, nnzb * nb * nb, "val"), (x, torch.float64, nrows * nb, "x"),
           (y, torch.float64, nrows * nb, "y")]
    for t, dt, ne, name in ops:
        _tensor_shape(t, dt, ne, name)
    for t, _, _, name in ops:
        _tensor_device(t, name, rowptr.device.index)
    ptr = [C.c_void_p(t.data_ptr()) for t, _, _, _ in ops]
    s = current_stream() if stream is None else stream
    _check(lib().fim_bsr_spmv(nrows, nb, *ptr, s), "fim_bsr_spmv")


def fim_ensemble_run(members, dt):
    """Advance the contexts `members` (Fim objects) together by dt.shape[1]
    steps each (fim_ensemble_run: one launch per kernel for all of them);
    dt[k, s] is step s of member k.  Returns (rc, status[count, nsteps],
    reports[count][nsteps])."""
    count = len(members)
    dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, np.float64), (count, np.shape(dt)[-1])))
    nsteps = dt.shape[1]
    handles = (C.c_void_p * max(count, 1))(*[m.h for m in members])
    status = np.zeros((count, nsteps), np.int32)
    reps = (FimStepReport * max(count * nsteps, 1))()
    rc = _check(lib().fim_ensemble_run(count, handles, nsteps, _p(dt, f64p), reps,
                                       _p(status, i32p)), "fim_ensemble_run")
    return rc, status, [[reps[k * nsteps + s] for s in range(nsteps)] for k in range(count)]


def fim_ensemble_tune(members, dt, trial_steps=1, cache_path=None):
    """Time trial steps of the batched ensemble with every candidate ILU(0)
    box, set the fastest on every member and cache it (fim_ensemble_tune).
    Returns (rc, report)."""
    count = len(members)
    handles = (C.c_void_p * max(count, 1))(*[m.h for m in members])
    rep = FimTuneReport()
    path = cache_path.encode() if cache_path else None
    rc = _check(lib().fim_ensemble_tune(count, handles, float(dt), int(trial_steps), path,
                                        C.byref(rep)), "fim_ensemble_tune")
    for m in members:
        m.options.tile = tuple(rep.box)
    return rc, rep
