"""Host-side checks of libexx.so that need no GPU.

* the library loads and exports every function declared in include/exx.h;
* argument validation returns the documented codes before any HIP call.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exx.h")

L = pytest.importorskip("paper_1712_07973_amd._lib")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(exx_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libexx.so is not built (run python -m paper_1712_07973_amd.build)")
    return L.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"


def test_version_and_error_strings(lib):
    assert lib.exx_version().decode().startswith("exx")
    assert lib.exx_error_string(0) == b"ok"
    assert lib.exx_error_string(-4) == b"workspace missing or too small"
    assert lib.exx_error_string(12345) == b"unknown error code"


def _grid(n=64, h=0.4, bc=1, kernel=0, R=0.0, omega=0.0, ny=None):
    g = L.ExxGrid()
    g.nx = n
    g.ny = n if ny is None else ny
    g.nz = n
    g.hx = g.hy = g.hz = h
    g.bc, g.kernel, g.R, g.omega = bc, kernel, R, omega
    return g


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), -1), (dict(h=-0.4), -1), (dict(h=float("nan")), -1), (dict(bc=7), -1),
    (dict(kernel=5), -1), (dict(kernel=1, omega=0.0, bc=0), -1), (dict(kernel=1, omega=0.2, bc=1), -1),
    (dict(n=44), -2), (dict(n=256), -2), (dict(n=64, ny=32), -2), (dict(n=24), -2),
])
def test_plan_validation_codes(lib, kw, code):
    h = C.c_void_p()
    g = _grid(**kw)
    rc = lib.exx_plan_create(C.byref(h), C.byref(g), 0, 16, 0)
    assert rc == code
    assert not h.value
    assert lib.exx_last_error()


def test_plan_validation_precision_and_counts(lib):
    h = C.c_void_p()
    g = _grid()
    assert lib.exx_plan_create(C.byref(h), C.byref(g), 9, 16, 0) == -1
    assert lib.exx_plan_create(C.byref(h), C.byref(g), 0, 0, 0) == -1
    assert lib.exx_plan_create(None, C.byref(g), 0, 16, 0) == -1
    g2 = _grid(n=112)
    assert lib.exx_plan_create(C.byref(h), C.byref(g2), 2, 16, 0) == -2  # FP64_FUSED n <= 96
    # the ISF kernel (2) is built for the free boundary only
    gp = _grid(bc=0)
    gp.kernel = 2
    assert lib.exx_plan_create(C.byref(h), C.byref(gp), 0, 16, 0) == -1
    assert b"ISF" in lib.exx_last_error()
    # plan flags: only EXX_PLAN_COMPLEX (1) is defined; batch flags: GRAPH (1),
    # COMPLEX (2), MERGE (4, FP32 only)
    assert lib.exx_plan_create(C.byref(h), C.byref(g), 0, 16, 2) == -1
    assert b"flags" in lib.exx_last_error()
    grids = (type(g) * 1)(g)
    counts = (C.c_int * 1)(4)
    assert lib.exx_batch_create(C.byref(h), grids, counts, 1, 0, 8) == -1
    assert not h.value
    assert b"batch flags" in lib.exx_last_error()
    assert lib.exx_batch_create(C.byref(h), grids, counts, 1, 2, 4) == -1
    assert not h.value
    assert b"FP32" in lib.exx_last_error()


def test_null_plan_calls(lib):
    size = C.c_size_t()
    assert lib.exx_workspace_bytes(None, 4, C.byref(size)) == -1
    assert lib.exx_compute(None, None, None, 1, 3, 0, None, None, None, None, 0, None) == -1
    assert lib.exx_plan_prepare(None, 4) == -1
    lib.exx_plan_destroy(None)  # no-op
    assert lib.exx_batch_create(None, None, None, 0, 0, 0) == -1
    assert lib.exx_compute_noalloc(None, None, None, 1, 3, 0, None, None, None, None) == -1
    assert lib.exx_gradient(None, None, None, 1, None, None, None, None, None, 0, None) == -1
    assert b"plan is NULL" in lib.exx_last_error()
    assert lib.exx_batch_autotune(None, None, None, 0, None, 0, None) == -1
    tun = L.ExxTuning()
    assert lib.exx_batch_get_tuning(None, 0, C.byref(tun)) == -1
