"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, its structs have the header's layout, and argument
validation rejects bad input before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2406_10862_amd import fim, reservoirs as rv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fim_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fim.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert sorted(fim.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "fim.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(fim_grid),sizeof(fim_rock),sizeof(fim_fluid),sizeof(fim_well),"
        "sizeof(fim_options),sizeof(fim_step_report),offsetof(fim_step_report,dt_sub),"
        "offsetof(fim_options,max_newton));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [C.sizeof(fim.FimGrid), C.sizeof(fim.FimRock), C.sizeof(fim.FimFluid),
            C.sizeof(fim.FimWell), C.sizeof(fim.FimOptions), C.sizeof(fim.FimStepReport),
            fim.FimStepReport.dt_sub.offset, fim.FimOptions.max_newton.offset]
    assert got == want


def _create(res, **opt_over):
    o = rv.Options()
    for k, v in opt_over.items():
        setattr(o, k, v)
    return fim.Fim(res, options=o, stream=C.c_void_p(0))


def _expect_arg_error(res, match, **opt_over):
    with pytest.raises(fim.FimError, match=match) as ei:
        _create(res, **opt_over)
    assert "(-1)" in str(ei.value)


def test_validation_rejects_bad_input_without_a_device():
    base = rv.config_c2_small(4, 4, 2)
    r = base.copy()
    r.fluid.p = r.fluid.p[::-1].copy()
    _expect_arg_error(r, "table pressures must increase")
    r = base.copy()
    r.wells[1].cells = np.array([0, 0], np.int32)
    _expect_arg_error(r, "duplicate cell")
    r = base.copy()
    r.wells[0].cells = np.array([10 ** 6], np.int32)
    _expect_arg_error(r, "out of range")
    r = base.copy()
    r.wells[1].control = rv.RATE
    _expect_arg_error(r, "rate-controlled producers")
    r = base.copy()
    r.poro[3] = 0.0
    _expect_arg_error(r, "porosity")
    _expect_arg_error(base, "restart", restart=0)
    _expect_arg_error(base, "restart", restart=41)
    _expect_arg_error(base, "mixed precision needs an ILU", precision=rv.MIXED,
                      precond=rv.PREC_CPR)
    _expect_arg_error(base, "unknown precision", precision=7)
    _expect_arg_error(base, "tile sizes", tile=(4, -1, 2))
    r = base.copy()
    r.wells.append(rv.Well(rv.INJ_GAS, rv.RATE, 10.0, np.array([5], np.int32)))
    _expect_arg_error(r, "gas injection needs model 3")
    bad = rv.blackoil_fluid()
    bad.bg = bad.bg * 1e-4        # makes the total compressibility negative
    r = rv.config_c1()
    r.fluid = bad
    _expect_arg_error(r, "negative total compressibility")


def test_spmv_rejects_bad_block_size_without_a_device():
    L = fim.lib()
    assert L.fim_bsr_spmv(4, 4, None, None, None, None, None, None) == fim.FIM_E_ARG
    assert b"nb must be 2 or 3" in L.fim_last_error()
    # an empty matrix is a no-op
    assert L.fim_bsr_spmv(0, 2, None, None, None, None, None, None) == fim.FIM_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(fim, "_LIB", None)
    monkeypatch.setattr(fim, "LIB_PATH", str(tmp_path / "libfim.so"))
    with pytest.raises(fim.FimError, match="no fallback"):
        fim.lib()


def test_ensemble_rejects_bad_arguments_without_a_device():
    L = fim.lib()
    # nothing to do is not an error
    assert L.fim_ensemble_run(0, None, 5, None, None, None) == fim.FIM_OK
    assert L.fim_ensemble_run(3, None, 0, None, None, None) == fim.FIM_OK
    assert L.fim_ensemble_run(-1, None, 1, None, None, None) == fim.FIM_E_ARG
    assert b"must be >= 0" in L.fim_last_error()
    assert L.fim_ensemble_run(2, None, 1, None, None, None) == fim.FIM_E_ARG
    assert b"required" in L.fim_last_error()


def _raw_create(nx, ny, nz, model=2, wells=()):
    """fim_create on a grid given by its dimensions only: one-element arrays
    stand in for every per-cell array, so the call must reject the size
    before it reads any of them."""
    L = fim.lib()
    one = (C.c_double * 1)(1.0)
    f64 = C.cast(one, fim.f64p)
    grid = fim.FimGrid(nx, ny, nz, f64, f64, f64, 0.0)
    rock = fim.FimRock(f64, f64, f64, f64, 0.0, 0.0)
    fl = rv.deadoil_fluid() if model == 2 else rv.blackoil_fluid()
    keep = [np.ascontiguousarray(a, np.float64) for a in (fl.p, fl.bo, fl.rs, fl.muo, fl.bg, fl.mug)]
    ptr = [a.ctypes.data_as(fim.f64p) for a in keep]
    fluid = fim.FimFluid(model=model, nrows=len(fl.p), p=ptr[0], bo=ptr[1], rs=ptr[2],
                         muo=ptr[3], bg=ptr[4], mug=ptr[5])
    wl = (fim.FimWell * max(len(wells), 1))(*wells)
    opt = fim.options_struct(rv.Options())
    h = C.c_void_p()
    rc = L.fim_create(C.byref(grid), C.byref(rock), C.byref(fluid), len(wells), wl,
                      C.byref(opt), C.c_void_p(0), C.byref(h))
    return rc, L.fim_last_error().decode(), h


def test_create_rejects_sizes_the_32_bit_indexing_cannot_address():
    # 2^28 cells
    rc, msg, h = _raw_create(1024, 1024, 256)
    assert rc == fim.FIM_E_ARG and "grid too large" in msg and not h.value
    # 10^8 cells: about 7*10^8 blocks, 2.8*10^9 values of 2x2 blocks
    rc, msg, h = _raw_create(1000, 1000, 100)
    assert rc == fim.FIM_E_ARG and "system too large" in msg and not h.value
    # 3x3 blocks reach the limit at fewer cells: 40M cells, 2.5*10^9 values
    rc, msg, h = _raw_create(400, 1000, 100, model=3)
    assert rc == fim.FIM_E_ARG and "system too large" in msg and not h.value
    # and the same grid with 2x2 blocks (1.1*10^9 values) passes the size
    # check, to fail on the first per-cell array instead
    rc, msg, h = _raw_create(400, 1000, 100, model=2)
    assert "system too large" not in msg


def test_device_tensor_checks_reject_bad_tensors_before_any_launch():
    torch = pytest.importorskip("torch")
    good = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(fim.FimError, match="dtype"):
        fim.dev_ptr(good.float(), torch.float64, 12, "P")
    with pytest.raises(fim.FimError, match="contiguous"):
        fim.dev_ptr(torch.zeros(12, 2, dtype=torch.float64)[:, 0], torch.float64, 12, "P")
    with pytest.raises(fim.FimError, match="elements"):
        fim.dev_ptr(good[:11], torch.float64, 12, "P")
    with pytest.raises(fim.FimError, match="GPU tensor"):
        fim.dev_ptr(good, torch.float64, 12, "P")
    with pytest.raises(fim.FimError, match="torch tensor"):
        fim.dev_ptr(np.zeros(12), torch.float64, 12, "P")
    # the SpMV wrapper checks every operand the same way
    rp = torch.zeros(5, dtype=torch.int32)
    ci = torch.zeros(3, dtype=torch.int32)
    with pytest.raises(fim.FimError, match="rowptr: dtype"):
        fim.fim_bsr_spmv(4, 2, rp.long(), ci, torch.zeros(12, dtype=torch.float64),
                         torch.zeros(8, dtype=torch.float64), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(fim.FimError, match="val: .*elements"):
        fim.fim_bsr_spmv(4, 2, rp, ci, torch.zeros(11, dtype=torch.float64),
                         torch.zeros(8, dtype=torch.float64), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(fim.FimError, match="GPU tensor"):
        fim.fim_bsr_spmv(4, 2, rp, ci, torch.zeros(12, dtype=torch.float64),
                         torch.zeros(8, dtype=torch.float64), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(fim.FimError, match="nb 4"):
        fim.fim_bsr_spmv(4, 4, rp, ci, None, None, None)


def test_tuner_rejects_bad_arguments_without_a_device():
    L = fim.lib()
    rep = fim.FimTuneReport()
    assert L.fim_ensemble_tune(0, None, 15.0, 1, None, C.byref(rep)) == fim.FIM_E_ARG
    assert b"members are required" in L.fim_last_error()
