"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/af.h, and validates its arguments."""
import ctypes as C
import os
import re

import pytest

from paper_2609_29081_amd import af
from paper_2609_29081_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "af.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    syms = declared_symbols()
    for name in ("af_init_grid", "af_set_bc", "af_rk_stage", "af_step", "af_run"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = af.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert sorted(af.EXPORTS) == sorted(declared_symbols())


def make(**kw):
    p = af.Params()
    assert af.lib().af_default_params(C.byref(p)) == af.AF_OK
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    st = af.lib().af_init_grid(C.byref(p), C.byref(h))
    return st, h


@pytest.mark.parametrize("field,value", [("dim", 3), ("n1", 3), ("n2", 2), ("gamma", 1.0),
                                         ("mu", -1e-3), ("Pr", 0.0), ("cfl_c", 0.0),
                                         ("cfl_v", -1.0), ("x1", 0.0), ("max_halvings", -1),
                                         ("limiter", 128), ("limiter", -1)])
def test_init_rejects_bad_parameters(field, value):
    st, h = make(**{field: value})
    assert st == af.AF_E_ARG
    assert af.lib().af_last_error()
    assert not h.value


@pytest.mark.parametrize("dim", [1, 2])
def test_init_takes_the_exact_pressure_rule(dim):
    st, h = make(dim=dim, n1=16, n2=8, limiter=af.LIM_ALL | af.LIM_PEXACT)
    assert st == af.AF_OK and h.value
    af.lib().af_destroy(h)


def test_sizes_match_the_documented_layout():
    for grid in (W.Grid(dim=2, n1=10, n2=7, bc=(W.PERIODIC, W.PERIODIC, W.NOSLIP, W.SYMMETRY)),
                 W.Grid(dim=2, n1=6, n2=9, bc=(W.OUTFLOW,) * 4),
                 W.Grid(dim=1, n1=12, bc=(W.PERIODIC,) * 4),
                 W.Grid(dim=1, n1=12, bc=(W.NOSLIP, W.OUTFLOW, 0, 0))):
        st, h = make(dim=grid.dim, n1=grid.n1, n2=grid.n2)
        assert st == af.AF_OK
        for side in range(2 if grid.dim == 1 else 4):
            assert af.lib().af_set_bc(h, side, grid.bc[side]) == af.AF_OK
        assert af.lib().af_state_len(h) == grid.state_len
        assert af.lib().af_state_bytes(h) == 8 * grid.state_len
        assert af.lib().af_workspace_bytes(h) > 8 * grid.state_len
        af.lib().af_destroy(h)


def test_bc_validation():
    st, h = make(dim=2, n1=8, n2=8)
    L = af.lib()
    assert L.af_set_bc(h, 4, 0) == af.AF_E_ARG
    assert L.af_set_bc(h, 0, 7) == af.AF_E_ARG
    assert L.af_set_bc(h, 0, af.PERIODIC) == af.AF_OK
    # one periodic side only: sizes are refused
    assert L.af_state_len(h) == 0
    assert L.af_set_bc(h, 1, af.PERIODIC) == af.AF_OK
    assert L.af_state_len(h) > 0
    L.af_destroy(h)
    st, h = make(dim=1, n1=8)
    assert L.af_set_bc(h, 2, 0) == af.AF_E_ARG
    L.af_destroy(h)


def test_stage_argument_checks_need_no_gpu():
    st, h = make(dim=2, n1=8, n2=8)
    L = af.lib()
    ws = C.c_void_p(256)
    assert L.af_rk_stage(h, 3, None, 1e-3, None, ws, C.c_void_p(512), ws, None) == af.AF_E_ARG
    assert L.af_rk_stage(h, 1, None, 1e-3, None, ws, C.c_void_p(512), ws, None) == af.AF_E_ARG
    assert L.af_rk_stage(h, 0, None, 1e-3, None, ws, ws, ws, None) == af.AF_E_ARG
    assert L.af_run(h, ws, ws, None, 0.0, 1.0, 5, 0, None, None) == af.AF_E_ARG
    L.af_destroy(h)
