"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, validates arguments before any device work, and its boundary-range
launch visits every ghost cell exactly once (section 2.4)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1504_02264_amd as les

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("les.h", "lesnet.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b((?:les|lesnet)_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_and_binding_agree():
    assert declared_functions() == sorted(les.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = les.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_default_params():
    p = les.default_params()
    assert p.omega == 1.8 and p.tol == 1e-5 and p.check_every == 4 and p.max_iter == 20000
    assert p.cs == 0.1 and p.nu == 1.5e-5 and p.alpha == -10.0 and p.beta == -1.0
    assert tuple(p.bc) == les.URBAN_BC
    assert les.lib().les_default_params(None) == les.LES_EINVAL


@pytest.mark.parametrize("grid,spacing,dt", [
    ((3, 8, 8), (1, 1, 1), 0.1),          # too small
    ((8, 8, 0), (1, 1, 1), 0.1),
    ((8, 8, 8), (0, 1, 1), 0.1),          # zero spacing
    ((8, 8, 8), (1, float("nan"), 1), 0.1),
    ((8, 8, 8), (1, 1, 1), 0.0),          # dt
    ((8, 8, 8), (1, 1, 1), float("inf")),
])
def test_create_rejects_bad_arguments(grid, spacing, dt):
    h = C.c_void_p()
    rc = les.lib().les_create(C.byref(les.Grid(*grid)), C.byref(les.Spacing(*spacing)), dt, None,
                              None, C.byref(h))
    assert rc == les.LES_EINVAL and not h.value


@pytest.mark.parametrize("field,val", [
    ("omega", 2.0), ("omega", 0.0), ("tol", -1.0), ("check_every", 0), ("max_iter", -1),
    ("cs", -0.1), ("nu", float("nan")), ("rebase_every", 0),
])
def test_create_rejects_bad_params(field, val):
    p = les.default_params(**{field: val})
    h = C.c_void_p()
    rc = les.lib().les_create(C.byref(les.Grid(8, 8, 8)), C.byref(les.Spacing(1, 1, 1)), 0.1,
                              None, C.byref(p), C.byref(h))
    assert rc == les.LES_EINVAL


@pytest.mark.parametrize("bc", [
    (les.OUTFLOW, les.OUTFLOW, 0, 0, 0, 0),   # outflow on x-
    (les.INFLOW, les.INFLOW, 0, 0, 0, 0),     # inflow on x+
    (les.INFLOW, les.OUTFLOW, les.INFLOW, 0, 0, 0),
    (les.INFLOW, les.OUTFLOW, 0, 0, 7, 0),
])
def test_create_rejects_bad_bc_sets(bc):
    p = les.default_params(bc=bc)
    h = C.c_void_p()
    rc = les.lib().les_create(C.byref(les.Grid(8, 8, 8)), C.byref(les.Spacing(1, 1, 1)), 0.1,
                              None, C.byref(p), C.byref(h))
    assert rc == les.LES_EINVAL


def _widths(n, v=1.0):
    return np.full(n, v, np.float64)


@pytest.mark.parametrize("bad", ["zero", "nan", "negative", "null", "singular", "small"])
def test_create_stretched_rejects_bad_arguments(bad):
    nx, ny, nz = 8, 6, 5
    hx, hy, hz = _widths(nx), _widths(ny), _widths(nz, 0.5)
    grid = les.Grid(nx, ny, nz)
    p = None
    if bad == "zero":
        hz[2] = 0.0
    elif bad == "nan":
        hy[1] = float("nan")
    elif bad == "negative":
        hx[7] = -1.0
    elif bad == "singular":   # stretched axes need the outflow face
        p = les.default_params(bc=(les.FREESLIP,) * 6)
    elif bad == "small":
        grid = les.Grid(3, ny, nz)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    args = [ptr(hx), None if bad == "null" else ptr(hy), ptr(hz)]
    rc = les.lib().les_create_stretched(C.byref(grid), *args, 0.05, None,
                                        None if p is None else C.byref(p), C.byref(h))
    assert rc == les.LES_EINVAL and not h.value


def test_null_handle_calls():
    L = les.lib()
    assert L.les_step(None, 1, None) == les.LES_EINVAL
    assert L.les_get_fields(None, None, None, None, None) == les.LES_EINVAL
    assert L.les_pressure_solve_noalloc(None, None, None, 1e-5, 10, None, None) == les.LES_EINVAL
    assert L.les_last_error(None) == b""
    L.les_destroy(None)
    # training-set preparation: argument checks come before any launch
    assert L.lesnet_crop(None, 4, 4, 4, 3, 0, 0, 0, 4, 4, 4, 0, None, None) == les.LES_EINVAL
    assert L.lesnet_gather(None, 8, 2, None, 1, None, None) == les.LES_EINVAL
    assert L.lesnet_sum_squares(None, 8, None, None) == les.LES_EINVAL
    assert L.lesnet_sum_squares(None, 0, None, None) == les.LES_EINVAL   # no output
    assert L.lesnet_scale_div(None, 8, 1.0, None, None) == les.LES_EINVAL


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 7, 4), (33, 17, 9), (64, 64, 32)])
def test_boundary_range_is_a_bijection(shape):
    """P13: the boundary-range items cover each ghost cell of the ghosted box
    exactly once (low and high side per item), and the padded tail maps to
    no cell."""
    nx, ny, nz = shape
    n = les.bc_range(nx, ny, nz)
    exact = (ny + 2) * (nz + 2) + nx * (nz + 2) + nx * ny
    assert n >= exact and n % 256 == 0 and n - exact < 256
    seen = np.zeros((nz + 2, ny + 2, nx + 2), np.int32)
    for item in range(n):
        f, a, b = les.bc_map(nx, ny, nz, item)
        if item >= exact:
            assert f == -1
            continue
        if f == 0:
            j, k = a, b
            seen[k, j, 0] += 1
            seen[k, j, nx + 1] += 1
        elif f == 1:
            i, k = a, b
            seen[k, 0, i] += 1
            seen[k, ny + 1, i] += 1
        else:
            i, j = a, b
            seen[0, j, i] += 1
            seen[nz + 1, j, i] += 1
    shell = np.ones_like(seen)
    shell[1:-1, 1:-1, 1:-1] = 0
    assert np.array_equal(seen, shell)
