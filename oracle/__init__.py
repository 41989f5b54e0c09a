"""FP64 CPU oracle of the urban-LES time step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It is the plain, slow, obviously
correct definition the GPU path is checked against and shares no code with
it (the GPU library lives in ``paper_1504_02264_amd``; neither imports the
other).

The C++ source (``les_oracle.cpp``) follows section 2 of the paper: the
per-step subroutine order (2.1), the tendency assembly from cov/diu pieces
(2.5.3), the red-black SOR update and colour order (2.6) and the boundary
face families (2.4).  Each function there names the reading it implements
where the paper is silent.

Arrays crossing this binding are float64, C order, i fastest, ghost-free:
``u[nz, ny, nx+1]``, ``v[nz, ny+1, nx]``, ``w[nz+1, ny, nx]`` and cell
arrays ``[nz, ny, nx]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "les_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

FREESLIP, NOSLIP, INFLOW, OUTFLOW = 0, 1, 2, 3
URBAN_BC = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, NOSLIP, FREESLIP)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain IEEE float64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-shared",
               "-fPIC", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OParams(C.Structure):
    _fields_ = [
        ("omega", C.c_double), ("tol", C.c_double),
        ("check_every", C.c_int32), ("max_iter", C.c_int32),
        ("cs", C.c_double), ("nu", C.c_double),
        ("alpha", C.c_double), ("beta", C.c_double),
        ("bc", C.c_int32 * 6), ("zero_guess", C.c_int32), ("pad_", C.c_int32),
    ]


class OStats(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("converged", C.c_int32),
        ("resid", C.c_double), ("rhs_norm", C.c_double), ("reltmp2", C.c_double),
        ("div_star", C.c_double), ("div_new", C.c_double), ("cfl", C.c_double),
        ("total_iters", C.c_int64), ("not_converged", C.c_int32), ("pad_", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                    C.c_double, P, C.POINTER(OParams)]
        L.oracle_create_stretched.restype = P
        L.oracle_create_stretched.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, C.c_double, P,
                                              C.POINTER(OParams)]
        L.oracle_destroy.argtypes = [P]
        L.oracle_set_inflow.argtypes = [P, P, C.c_double, C.c_uint64]
        L.oracle_set_inflow_pair.argtypes = [P, C.c_double, P, C.c_double, P]
        L.oracle_step.argtypes = [P, C.c_int, P, P, C.POINTER(OStats)]
        L.oracle_set_fields.argtypes = [P, P, P, P, P, C.c_int]
        L.oracle_get_fields.argtypes = [P, P, P, P, P]
        L.oracle_get_ghosted.argtypes = [P, P, P, P]
        L.oracle_get_aux.argtypes = [P, C.c_int, P, P, P]
        L.oracle_nut.argtypes = [P, P, P, P, P]
        L.oracle_force.argtypes = [P, P, P, P, P, P, P]
        L.oracle_divergence.argtypes = [P, P, P, P, P]
        L.oracle_project.argtypes = [P, P, P, P, P]
        L.oracle_apply_A.argtypes = [P, P, P]
        L.oracle_pressure_solve.argtypes = [P, P, P, C.c_double, C.c_int, C.c_int,
                                            C.POINTER(OStats)]
        L.oracle_sor_iterations.restype = C.c_double
        L.oracle_sor_iterations.argtypes = [P, P, P, C.c_int]
        L.oracle_twinned_iterations.argtypes = [P, P, P, C.c_double, C.c_int]
        L.oracle_residual.restype = C.c_double
        L.oracle_residual.argtypes = [P, P, P]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64]
        L.oracle_inflow_value.restype = C.c_double
        L.oracle_inflow_value.argtypes = [P, C.c_int, C.c_int, C.c_int64]
        _lib = L
    return _lib


def default_params(**kw) -> OParams:
    p = OParams()
    p.omega, p.tol, p.check_every, p.max_iter = 1.8, 1e-5, 4, 20000
    p.cs, p.nu, p.alpha, p.beta = 0.1, 1.5e-5, -10.0, -1.0
    for f, b in enumerate(URBAN_BC):
        p.bc[f] = b
    p.zero_guess = 0
    for k, v in kw.items():
        if k == "bc":
            for f, b in enumerate(v):
                p.bc[f] = b
        else:
            setattr(p, k, v)
    return p


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """One FP64 LES instance (see module docstring for the array layout)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, dt, mask=None, params: Optional[OParams] = None,
                 **kw):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dx, self.dy, self.dz, self.dt = dx, dy, dz, dt
        self.params = params if params is not None else default_params(**kw)
        self._mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        if self._mask is not None:
            assert self._mask.shape == (nz, ny, nx)
        # dx, dy, dz: a uniform spacing, or the nx / ny / nz cell widths of a
        # stretched axis (the paper's 1-D spacing arrays)
        self.hx, self.hy, self.hz = (np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (n,)))
                                     for h, n in ((dx, nx), (dy, ny), (dz, nz)))
        self.stretched = any(np.ndim(h) > 0 for h in (dx, dy, dz))
        if self.stretched:
            self.h = lib().oracle_create_stretched(nx, ny, nz, _ptr(self.hx), _ptr(self.hy),
                                                   _ptr(self.hz), dt, _ptr(self._mask),
                                                   C.byref(self.params))
        else:
            self.h = lib().oracle_create(nx, ny, nz, dx, dy, dz, dt, _ptr(self._mask),
                                         C.byref(self.params))
        if not self.h:
            raise ValueError("oracle_create rejected its arguments")
        self.last_iters = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().oracle_destroy(h)
            self.h = None

    # shapes
    @property
    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)

    def set_inflow(self, profile, amp=0.01, seed=0):
        prof = np.ascontiguousarray(profile, dtype=np.float32)
        assert prof.shape == (self.nz,)
        lib().oracle_set_inflow(self.h, _ptr(prof), float(amp), int(seed))

    def set_inflow_pair(self, t0, prof0, t1, prof1):
        """Linear interpolation in time between two inflow profile samples
        (section 4, coupled time loop), from the next step on."""
        a = np.ascontiguousarray(prof0, dtype=np.float32)
        b = np.ascontiguousarray(prof1, dtype=np.float32)
        assert a.shape == (self.nz,) and b.shape == (self.nz,)
        rc = lib().oracle_set_inflow_pair(self.h, float(t0), _ptr(a), float(t1), _ptr(b))
        if rc != 0:
            raise ValueError("oracle_set_inflow_pair: set_inflow first, and t0 < t1")

    def step(self, n=1, forced: Optional[Sequence[int]] = None):
        st = OStats()
        iters = np.zeros(max(n, 1), dtype=np.int32)
        f = None if forced is None else np.ascontiguousarray(forced, dtype=np.int32)
        if f is not None:
            assert f.shape[0] >= n
        rc = lib().oracle_step(self.h, n, _ptr(f), _ptr(iters), C.byref(st))
        self.last_iters = iters[:n].copy()
        return rc, st.as_dict()

    def set_fields(self, u=None, v=None, w=None, p=None, reset_history=True):
        su, sv, sw, sp = self.shapes
        a = [None if x is None else _f64(x) for x in (u, v, w, p)]
        for x, s in zip(a, (su, sv, sw, sp)):
            if x is not None:
                assert x.shape == s, (x.shape, s)
        lib().oracle_set_fields(self.h, *[_ptr(x) for x in a], int(reset_history))

    def get_fields(self):
        su, sv, sw, sp = self.shapes
        u, v, w, p = (np.zeros(s) for s in (su, sv, sw, sp))
        lib().oracle_get_fields(self.h, _ptr(u), _ptr(v), _ptr(w), _ptr(p))
        return u, v, w, p

    def get_ghosted(self):
        s = (self.nz + 2, self.ny + 2, self.nx + 2)
        u, v, w = np.zeros(s), np.zeros(s), np.zeros(s)
        lib().oracle_get_ghosted(self.h, _ptr(u), _ptr(v), _ptr(w))
        return u, v, w

    def get_nut(self):
        a = np.zeros(self.shapes[3])
        lib().oracle_get_aux(self.h, 0, _ptr(a), None, None)
        return a

    def get_rhs(self):
        a = np.zeros(self.shapes[3])
        lib().oracle_get_aux(self.h, 1, _ptr(a), None, None)
        return a

    def get_force(self):
        su, sv, sw, _ = self.shapes
        a, b, c = np.zeros(su), np.zeros(sv), np.zeros(sw)
        lib().oracle_get_aux(self.h, 2, _ptr(a), _ptr(b), _ptr(c))
        return a, b, c

    def get_usum(self):
        su, sv, sw, _ = self.shapes
        a, b, c = np.zeros(su), np.zeros(sv), np.zeros(sw)
        lib().oracle_get_aux(self.h, 3, _ptr(a), _ptr(b), _ptr(c))
        return a, b, c

    # ---- stage-level calls on caller data
    def nut_of(self, u, v, w):
        out = np.zeros(self.shapes[3])
        lib().oracle_nut(self.h, _ptr(_f64(u)), _ptr(_f64(v)), _ptr(_f64(w)), _ptr(out))
        return out

    def force_of(self, u, v, w):
        su, sv, sw, _ = self.shapes
        a, b, c = np.zeros(su), np.zeros(sv), np.zeros(sw)
        lib().oracle_force(self.h, _ptr(_f64(u)), _ptr(_f64(v)), _ptr(_f64(w)),
                           _ptr(a), _ptr(b), _ptr(c))
        return a, b, c

    def divergence(self, u, v, w):
        out = np.zeros(self.shapes[3])
        lib().oracle_divergence(self.h, _ptr(_f64(u)), _ptr(_f64(v)), _ptr(_f64(w)), _ptr(out))
        return out

    def project(self, u, v, w, p):
        u, v, w = _f64(u).copy(), _f64(v).copy(), _f64(w).copy()
        lib().oracle_project(self.h, _ptr(u), _ptr(v), _ptr(w), _ptr(_f64(p)))
        return u, v, w

    def apply_A(self, p):
        out = np.zeros(self.shapes[3])
        lib().oracle_apply_A(self.h, _ptr(_f64(p)), _ptr(out))
        return out

    def pressure_solve(self, rhs, p0=None, tol=1e-5, max_iter=20000, forced=-1):
        p = np.zeros(self.shapes[3]) if p0 is None else _f64(p0).copy()
        st = OStats()
        rc = lib().oracle_pressure_solve(self.h, _ptr(_f64(rhs)), _ptr(p), float(tol),
                                         int(max_iter), int(forced), C.byref(st))
        return p, st.as_dict(), rc

    def sor_iterations(self, rhs, p0, n):
        p = _f64(p0).copy()
        s = lib().oracle_sor_iterations(self.h, _ptr(_f64(rhs)), _ptr(p), int(n))
        return p, s

    def twinned_iterations(self, rhs, p0, omega, n):
        """n iterations of twinned double buffering (section 2.6): each half
        updates every cell from the other buffer (relaxed Jacobi)."""
        p = _f64(p0).copy()
        lib().oracle_twinned_iterations(self.h, _ptr(_f64(rhs)), _ptr(p), float(omega), int(n))
        return p

    def residual(self, rhs, p):
        return lib().oracle_residual(self.h, _ptr(_f64(rhs)), _ptr(_f64(p)))

    def inflow_value(self, j, k, step):
        """1-based j, k."""
        return lib().oracle_inflow_value(self.h, j, k, step)


def splitmix64(x: int) -> int:
    return int(lib().oracle_splitmix64(x))
