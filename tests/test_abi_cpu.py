"""Host-side checks of the C ABI (no GPU): symbols, defaults, validation.

Invalid arguments are rejected before any device access, so these calls
run without a GPU.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rexi.h")


@pytest.fixture(scope="module")
def rx():
    from paper_1912_03312_amd import rexi
    return rexi


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rexi_[a-z_A-Z]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rexi_setup", "rexi_apply_H", "rexi_step", "rexi_step_adjoint", "rexi_setup_batch", "rexi_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(rx):
    lib = C.CDLL(rx.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(rx.EXPORTS) == set(declared_functions())


def test_status_strings_and_defaults(rx):
    assert rx.status_string(0) == "REXI_OK"
    assert rx.status_string(4) == "REXI_E_NOT_CONVERGED"
    o = rx.default_options()
    assert o.m == 30 and o.max_cycles == 40 and o.tol == 1e-10 and o.reorth == 1 and o.inner_rtol == 0.1
    assert o.precision == rx.PREC_C128 and o.solver == rx.SOLVER_PER_POLE


def _setup_raw(rx, grid, hbar=1.0, mass=1.0, dt=0.1, K=1, sigma=(5 + 1j,), beta=(1 + 0j,), opt=None, vptr=8):
    raw = rx._H()
    o = opt if opt is not None else rx.default_options()
    st = rx._lib.rexi_setup(C.byref(raw), C.byref(grid), C.c_void_p(vptr), hbar, mass, dt, K,
                            rx._c128_array(sigma), rx._c128_array(beta), C.byref(o), None)
    buf = C.create_string_buffer(256)
    rx._lib.rexi_last_error(None, buf, 256)
    return st, buf.value.decode()


@pytest.mark.parametrize("case", [
    dict(grid=dict(n=(0,), lo=(0,), hi=(1,))),
    dict(grid=dict(n=(4,), lo=(1,), hi=(1,))),
    dict(grid=dict(n=(4, 4, 4, 4), lo=(0,) * 4, hi=(1,) * 4)),
    dict(hbar=0.0), dict(hbar=-1.0), dict(mass=0.0), dict(dt=0.0), dict(dt=float("inf")),
    dict(K=0), dict(sigma=(float("nan"),)), dict(beta=(complex(0, float("inf")),)),
])
def test_invalid_arguments_are_rejected_without_device(rx, case):
    g = case.get("grid", dict(n=(8,), lo=(0.0,), hi=(1.0,)))
    if len(g["n"]) > 3:
        grid = rx.make_grid((4,), (0,), (1,))
        grid.ndim = 4
    else:
        grid = rx.make_grid(g["n"], g["lo"], g["hi"])
    kw = {k: v for k, v in case.items() if k != "grid"}
    st, msg = _setup_raw(rx, grid, **kw)
    assert st == rx.REXI_E_INVALID_ARG, msg
    assert msg


@pytest.mark.parametrize("field,value", [("m", 0), ("m", 257), ("reorth_eta", 0.0), ("reorth_eta", 1.0), ("solver", 5), ("max_cycles", 0), ("tol", -1.0),
                                         ("precision", 7), ("reorth", 3), ("inner_rtol", 1.5),
                                         ("march_planes", -2), ("march_planes", 1025), ("march_slots", 4),
                                         ("march_slots", 1), ("march_slots", 6), ("march_slots", -1),
                                         ("fallback", 3), ("fallback", -1), ("fallback_m", 0), ("fallback_m", 257),
                                         ("fallback_bytes", -1), ("stab_eps", -0.1), ("stab_eps", 1.0),
                                         ("stab_eps", float("nan")), ("center", 2)])
def test_invalid_options(rx, field, value):
    o = rx.default_options()
    setattr(o, field, value)
    st, msg = _setup_raw(rx, rx.make_grid((8,), (0,), (1,)), opt=o)
    assert st == rx.REXI_E_INVALID_ARG, msg


def test_null_pointers(rx):
    assert rx._lib.rexi_setup(None, None, None, 1.0, 1.0, 1.0, 1, None, None, None, None) == rx.REXI_E_INVALID_ARG
    assert rx._lib.rexi_step(None, None, None, 1, None, None) == rx.REXI_E_INVALID_ARG
    assert rx._lib.rexi_destroy(None) == rx.REXI_OK
    assert rx._lib.rexi_tiling_info(None, None) == rx.REXI_E_INVALID_ARG


def test_shifted_solver_option_constraints(rx):
    o = rx.default_options(solver="shifted", precision="c64")
    st, msg = _setup_raw(rx, rx.make_grid((8,), (0,), (1,)), opt=o)
    assert st == rx.REXI_E_INVALID_ARG and "complex128" in msg
    # Q1 elements on the shared basis: one instance, fallback 0 or 1
    o = rx.default_options(solver="shifted", discretization="fem", fallback=2)
    st, msg = _setup_raw(rx, rx.make_grid((8,), (0,), (1,)), opt=o)
    assert st == rx.REXI_E_INVALID_ARG and "fallback" in msg
    o = rx.default_options(solver="shifted", discretization="fem")
    G = (rx.Grid * 2)(rx.make_grid((8,), (0,), (1,)), rx.make_grid((6,), (0,), (1,)))
    dbl = (C.c_double * 2)(1.0, 1.0)
    Ks = (C.c_int32 * 2)(1, 1)
    raw = rx._H()
    st = rx._lib.rexi_setup_batch(C.byref(raw), 2, G, C.c_void_p(8), dbl, dbl, (C.c_double * 2)(0.1, 0.1), Ks,
                                  rx._c128_array((5 + 1j, 5 + 1j)), rx._c128_array((1 + 0j, 1 + 0j)), C.byref(o),
                                  None)
    buf = C.create_string_buffer(256)
    rx._lib.rexi_last_error(None, buf, 256)
    assert st == rx.REXI_E_INVALID_ARG and "one instance" in buf.value.decode()
    o = rx.default_options(discretization=2)
    st, msg = _setup_raw(rx, rx.make_grid((8,), (0,), (1,)), opt=o)
    assert st == rx.REXI_E_INVALID_ARG
