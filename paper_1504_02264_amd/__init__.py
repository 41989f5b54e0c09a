"""Thin Python binding of the MI355X urban-LES library (``libles.so``).

Argument marshalling only: every step of the time step runs in the HIP
kernels behind the C ABI declared in ``include/les.h``.  The names follow
that header (``les_create`` -> :class:`LES`, ``les_step`` -> :meth:`LES.step`
...).  There is no CPU fallback: importing works without a GPU, but any
call that reaches the library fails loudly if ``libles.so`` is missing or
no HIP device is present.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAPER_1504_02264_AMD_LIB points the binding at another build of the same
# library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("PAPER_1504_02264_AMD_LIB") or os.path.join(_HERE, "libles.so")

LES_OK, LES_NOT_CONVERGED = 0, 1
LES_EINVAL, LES_ENOMEM, LES_EDEVICE, LES_ENONFINITE, LES_ESTATE = -1, -2, -3, -4, -5
FREESLIP, NOSLIP, INFLOW, OUTFLOW = 0, 1, 2, 3
URBAN_BC = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, NOSLIP, FREESLIP)

# every function include/les.h and include/lesnet.h declare
EXPORTS = (
    "les_default_params", "les_create", "les_create_stretched", "les_destroy", "les_last_error",
    "les_set_stream",
    "les_set_inflow", "les_set_inflow_pair", "les_step", "les_pressure_solve", "les_pressure_solve_dev",
    "les_pressure_solve_noalloc",
    "les_pressure_solve_twinned",
    "les_get_fields", "les_get_fields_dev", "les_set_fields", "les_get_aux", "les_get_ghosted",
    "les_get_step", "les_state_size", "les_get_state", "les_set_state", "les_bc_range",
    "les_bc_map", "les_get_timing", "les_autotune", "les_set_sor_variant",
    "les_ensemble_create", "les_ensemble_step", "les_ensemble_autotune",
    "les_ensemble_last_error", "les_ensemble_destroy", "les_ensemble_set_mode",
    "les_ensemble_set_variant",
    "les_ensemble_tuning", "les_set_initial_guess_dev",
    # include/lesnet.h
    "lesnet_default_config", "lesnet_create", "lesnet_destroy", "lesnet_last_error",
    "lesnet_num_params", "lesnet_get_params", "lesnet_set_params", "lesnet_get_grads",
    "lesnet_forward", "lesnet_gradients", "lesnet_train_step", "lesnet_set_lr", "lesnet_op", "les_warm_grid",
    "les_set_warm_start", "les_set_capture", "lesnet_crop", "lesnet_gather", "lesnet_sum_squares",
    "lesnet_scale_div",
)
ENSEMBLE_BATCHED, ENSEMBLE_PERSISTENT = 0, 1
NUM_SOR_VARIANTS = 14
# (row width TX, planes per block KT) of each half-sweep variant, and
# (TX, KT, wavefronts per block) of the fused red-black variants 8-11 (KT 0:
# chosen per grid); 12-13 run two iterations per launch (64 lanes x 32
# rows; KT: the resident blocks per compute unit the plane count is chosen
# for), as in the library
SOR_VARIANTS = ((64, 1), (32, 1), (64, 2), (32, 2), (64, 4), (32, 4), (64, 8), (32, 8),
                (32, 12, 16), (64, 16, 16), (32, 0, 16), (64, 0, 16), (64, 1, 16), (64, 2, 16))
NUM_SPLIT_SOR_VARIANTS = 8
FIRST_TWO_ITER_SOR_VARIANT = 12
KERNEL_NAMES = ("nut", "tendency", "inflow", "rhs", "sor", "check", "rebase", "project", "bc")


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * len(KERNEL_NAMES)), ("launches", C.c_int64 * len(KERNEL_NAMES))]


class LesError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"LES error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Spacing(C.Structure):
    _fields_ = [("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("omega", C.c_double), ("tol", C.c_double),
        ("check_every", C.c_int32), ("max_iter", C.c_int32),
        ("cs", C.c_double), ("nu", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
        ("bc", C.c_int32 * 6), ("zero_guess", C.c_int32), ("rebase_every", C.c_int32),
        ("diagnostics", C.c_int32), ("timing", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [
        ("steps", C.c_int32), ("not_converged", C.c_int32), ("sor_iters_total", C.c_int64),
        ("sor_iters_last", C.c_int32), ("pad_", C.c_int32),
        ("resid_last", C.c_double), ("reltmp2_last", C.c_double), ("rhs_norm_last", C.c_double),
        ("div_star_last", C.c_double), ("div_new_last", C.c_double), ("cfl_last", C.c_double),
        ("ms_total", C.c_double), ("iters_out", C.POINTER(C.c_int32)),
        ("warm_taken", C.c_int32), ("pad2_", C.c_int32),
        ("warm_r_prev_last", C.c_double), ("warm_r_net_last", C.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_
                if f not in ("pad_", "pad2_", "iters_out")}


class NetConfig(C.Structure):
    _fields_ = [("c1", C.c_int32), ("c2", C.c_int32), ("c3", C.c_int32), ("pad_", C.c_int32),
                ("seed", C.c_uint64), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("resid", C.c_double),
                ("rhs_norm", C.c_double), ("reltmp2", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EnsembleStats(C.Structure):
    _fields_ = [("members", C.c_int32), ("steps", C.c_int32), ("cells_total", C.c_int64),
                ("sor_iters_total", C.c_int64), ("not_converged", C.c_int32), ("pad_", C.c_int32),
                ("ms_total", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


_lib = None


def lib():
    """Load ``libles.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1504_02264_amd.build` (no CPU fallback exists)")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes this library bind to that one runtime, so device pointers
    # and streams from torch are valid here
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.les_default_params.argtypes = [C.POINTER(Params)]
    L.les_create.argtypes = [C.POINTER(Grid), C.POINTER(Spacing), C.c_double, P,
                             C.POINTER(Params), C.POINTER(P)]
    L.les_destroy.argtypes = [P]
    L.les_destroy.restype = None
    L.les_last_error.argtypes = [P]
    L.les_last_error.restype = C.c_char_p
    L.les_set_stream.argtypes = [P, P]
    L.les_create_stretched.argtypes = [C.POINTER(Grid), P, P, P, C.c_double, P, C.POINTER(Params),
                                       C.POINTER(C.c_void_p)]
    L.les_set_inflow.argtypes = [P, P, C.c_float, C.c_uint64]
    L.les_set_inflow_pair.argtypes = [P, C.c_double, P, C.c_double, P]
    L.les_step.argtypes = [P, C.c_int32, C.POINTER(StepStats)]
    L.les_pressure_solve.argtypes = [P, P, P, C.c_double, C.c_int32, C.POINTER(SolveStats)]
    L.les_pressure_solve_dev.argtypes = [P, P, P, C.c_double, C.c_int32, C.POINTER(SolveStats), P]
    L.les_pressure_solve_noalloc.argtypes = [P, P, P, C.c_double, C.c_int32, C.POINTER(SolveStats), P]
    L.les_pressure_solve_twinned.argtypes = [P, P, P, C.c_double, C.c_int32,
                                             C.POINTER(SolveStats), C.POINTER(C.c_double), P]
    L.les_get_fields.argtypes = [P, P, P, P, P]
    L.les_get_fields_dev.argtypes = [P, P, P, P, P, P]
    L.les_set_fields.argtypes = [P, P, P, P, P, C.c_int32]
    L.les_get_aux.argtypes = [P, C.c_int32, P, P, P]
    L.les_set_initial_guess_dev.argtypes = [P, P, P]
    L.les_get_ghosted.argtypes = [P, P, P, P]
    L.les_get_step.argtypes = [P, C.POINTER(C.c_int64)]
    L.les_state_size.argtypes = [P, C.POINTER(C.c_int64)]
    L.les_get_state.argtypes = [P, P, C.c_int64]
    L.les_set_state.argtypes = [P, P, C.c_int64]
    L.les_get_timing.argtypes = [P, C.POINTER(Timing), C.c_int32]
    L.les_autotune.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), P]
    L.les_set_sor_variant.argtypes = [P, C.c_int32]
    L.les_ensemble_create.argtypes = [C.c_int32, C.POINTER(P), C.POINTER(P)]
    L.les_ensemble_step.argtypes = [P, C.c_int32, C.POINTER(EnsembleStats), P]
    L.les_ensemble_autotune.argtypes = [P, C.c_int32]
    L.les_ensemble_last_error.argtypes = [P]
    L.les_ensemble_last_error.restype = C.c_char_p
    L.les_ensemble_set_mode.argtypes = [P, C.c_int32]
    L.les_ensemble_set_variant.argtypes = [P, C.c_int32]
    L.les_ensemble_tuning.argtypes = [P, C.POINTER(C.c_int32), P]
    L.les_ensemble_destroy.argtypes = [P]
    L.les_ensemble_destroy.restype = None
    L.les_bc_range.argtypes = [C.POINTER(Grid)]
    L.les_bc_range.restype = C.c_int64
    L.les_bc_map.argtypes = [C.POINTER(Grid), C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32)]
    L.lesnet_default_config.argtypes = [C.POINTER(NetConfig)]
    L.lesnet_create.argtypes = [C.POINTER(NetConfig), C.POINTER(P)]
    L.lesnet_destroy.argtypes = [P]
    L.lesnet_destroy.restype = None
    L.lesnet_last_error.argtypes = [P]
    L.lesnet_last_error.restype = C.c_char_p
    L.lesnet_num_params.argtypes = [P, C.POINTER(C.c_int64)]
    for f in ("lesnet_get_params", "lesnet_set_params", "lesnet_get_grads"):
        getattr(L, f).argtypes = [P, P, C.c_int64]
    I = C.c_int32
    L.lesnet_forward.argtypes = [P, I, I, I, I, P, P, P]
    L.lesnet_gradients.argtypes = [P, I, I, I, I, P, P, P]
    L.lesnet_train_step.argtypes = [P, I, I, I, I, P, P, C.POINTER(C.c_double), P]
    L.lesnet_set_lr.argtypes = [P, C.c_double]
    L.lesnet_op.argtypes = [I, I, I, I, I, I, I, P, P, P, P, P]
    L.les_warm_grid.argtypes = [P, C.POINTER(I), C.POINTER(I), C.POINTER(I)]
    L.les_set_warm_start.argtypes = [P, P, C.c_double, C.c_int32, C.c_int32, C.c_int32]
    L.les_set_capture.argtypes = [P, P, P, C.c_int32]
    L.lesnet_crop.argtypes = [P, I, I, I, I, I, I, I, I, I, I, I, P, P]
    L.lesnet_gather.argtypes = [P, C.c_int64, C.c_int64, P, I, P, P]
    L.lesnet_sum_squares.argtypes = [P, C.c_int64, P, P]
    L.lesnet_scale_div.argtypes = [P, C.c_int64, C.c_float, P, P]
    _lib = L
    return L


def default_params(**kw) -> Params:
    p = Params()
    lib().les_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "bc":
            for f, b in enumerate(v):
                p.bc[f] = b
        else:
            setattr(p, k, v)
    return p


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _current_stream() -> int:
    """torch's current HIP stream on the current device (its raw handle)."""
    import torch
    return torch.cuda.current_stream().cuda_stream


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class LES:
    """One LES instance on the current HIP device (``les_create``)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, dt, mask=None, params: Optional[Params] = None,
                 **kw):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dt = float(dt)
        self.params = params if params is not None else default_params(**kw)
        m = None
        if mask is not None:
            m = np.ascontiguousarray(mask, dtype=np.uint8)
            if m.shape != (nz, ny, nx):
                raise ValueError("mask must be [nz, ny, nx]")
        h = C.c_void_p()
        # dx, dy, dz: uniform spacings, or (any of them) the cell widths of a
        # stretched axis -> les_create_stretched with all three width arrays
        self.stretched = any(np.ndim(d) > 0 for d in (dx, dy, dz))
        if self.stretched:
            self.widths = tuple(np.ascontiguousarray(np.broadcast_to(np.asarray(d, np.float64), (n,)))
                                for d, n in ((dx, self.nx), (dy, self.ny), (dz, self.nz)))
            rc = lib().les_create_stretched(C.byref(Grid(nx, ny, nz)), *(_ptr(w) for w in self.widths),
                                            dt, _ptr(m), C.byref(self.params), C.byref(h))
        else:
            rc = lib().les_create(C.byref(Grid(nx, ny, nz)), C.byref(Spacing(dx, dy, dz)), dt,
                                  _ptr(m), C.byref(self.params), C.byref(h))
        if rc != LES_OK:
            raise LesError(rc, "les_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().les_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, rc, ok=(LES_OK,)):
        if rc not in ok:
            raise LesError(rc, lib().les_last_error(self.h).decode())
        return rc

    @property
    def shapes(self):
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx), (nz, ny, nx)

    def set_stream(self, stream_handle: int):
        return self._check(lib().les_set_stream(self.h, C.c_void_p(stream_handle)))

    def set_inflow(self, profile, noise_amp=0.01, seed=0):
        prof = _f32(profile, (self.nz,))
        return self._check(lib().les_set_inflow(self.h, _ptr(prof), float(noise_amp), int(seed)))

    def set_inflow_pair(self, t0, prof0, t1, prof1):
        """Interpolate the inflow profile in time between (t0, prof0) and
        (t1, prof1) from the next step on (les_set_inflow_pair)."""
        a = _f32(prof0, (self.nz,))
        b = _f32(prof1, (self.nz,))
        return self._check(lib().les_set_inflow_pair(self.h, float(t0), _ptr(a), float(t1), _ptr(b)))

    def step(self, n=1, allow_not_converged=True):
        """Advance n steps; returns (status, stats dict, per-step SOR iterations)."""
        st = StepStats()
        iters = np.zeros(max(int(n), 1), dtype=np.int32)
        st.iters_out = iters.ctypes.data_as(C.POINTER(C.c_int32))
        ok = (LES_OK, LES_NOT_CONVERGED) if allow_not_converged else (LES_OK,)
        rc = self._check(lib().les_step(self.h, int(n), C.byref(st)), ok)
        return rc, st.as_dict(), iters[:n].copy()

    def pressure_solve(self, rhs, p0=None, tol=1e-5, max_iter=20000):
        sc = self.shapes[3]
        r = _f32(rhs, sc)
        p = np.zeros(sc, np.float32) if p0 is None else _f32(p0, sc).copy()
        st = SolveStats()
        rc = self._check(lib().les_pressure_solve(self.h, _ptr(r), _ptr(p), float(tol),
                                                  int(max_iter), C.byref(st)),
                         (LES_OK, LES_NOT_CONVERGED))
        return p, st.as_dict(), rc

    def pressure_solve_dev(self, d_rhs, d_p, tol=1e-5, max_iter=20000, stream=None):
        """Device-pointer solve; d_rhs / d_p are contiguous float32 torch
        tensors.  Ordered on `stream` (default: torch's current stream, so
        the caller's earlier and later torch work on them is ordered)."""
        st = SolveStats()
        s = C.c_void_p(_current_stream() if stream is None else stream)
        rc = self._check(lib().les_pressure_solve_dev(self.h, C.c_void_p(d_rhs.data_ptr()),
                                                      C.c_void_p(d_p.data_ptr()), float(tol),
                                                      int(max_iter), C.byref(st), s),
                         (LES_OK, LES_NOT_CONVERGED))
        return st.as_dict(), rc

    def pressure_solve_noalloc(self, d_rhs, d_p, tol=1e-5, max_iter=20000, stream=None):
        """les_pressure_solve_noalloc: the device-pointer solve on the
        library's static workspace (no device allocation); arguments and
        ordering as pressure_solve_dev."""
        st = SolveStats()
        s = C.c_void_p(_current_stream() if stream is None else stream)
        rc = self._check(lib().les_pressure_solve_noalloc(self.h, C.c_void_p(d_rhs.data_ptr()),
                                                          C.c_void_p(d_p.data_ptr()), float(tol),
                                                          int(max_iter), C.byref(st), s),
                         (LES_OK, LES_NOT_CONVERGED))
        return st.as_dict(), rc

    def pressure_solve_twinned(self, d_rhs, d_p, omega=1.0, iters=50, stream=None):
        """Twinned double-buffer relaxation (les_pressure_solve_twinned) on
        contiguous float32 device tensors, ordered on `stream` (default:
        torch's current stream); returns (stats, ms of the sweeps)."""
        st = SolveStats()
        ms = C.c_double(0.0)
        s = C.c_void_p(_current_stream() if stream is None else stream)
        self._check(lib().les_pressure_solve_twinned(self.h, C.c_void_p(d_rhs.data_ptr()),
                                                     C.c_void_p(d_p.data_ptr()), float(omega),
                                                     int(iters), C.byref(st), C.byref(ms), s))
        return st.as_dict(), ms.value

    def get_fields(self):
        su, sv, sw, sp = self.shapes
        u, v, w, p = (np.zeros(s, np.float32) for s in (su, sv, sw, sp))
        self._check(lib().les_get_fields(self.h, _ptr(u), _ptr(v), _ptr(w), _ptr(p)))
        return u, v, w, p

    def get_fields_dev(self, d_u, d_v, d_w, d_p, stream=None):
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        s = None if stream is None else C.c_void_p(stream)
        return self._check(lib().les_get_fields_dev(self.h, ptr(d_u), ptr(d_v), ptr(d_w),
                                                    ptr(d_p), s))

    def set_fields(self, u=None, v=None, w=None, p=None, reset_history=True):
        su, sv, sw, sp = self.shapes
        a = [None if x is None else _f32(x, s) for x, s in zip((u, v, w, p), (su, sv, sw, sp))]
        return self._check(lib().les_set_fields(self.h, *[_ptr(x) for x in a],
                                                int(bool(reset_history))))

    def set_initial_guess_dev(self, d_p, stream=None):
        """Start the next solve from the device tensor d_p [nz, ny, nx]."""
        s = None if stream is None else C.c_void_p(stream)
        return self._check(lib().les_set_initial_guess_dev(self.h, C.c_void_p(d_p.data_ptr()), s))

    def get_nut(self):
        a = np.zeros(self.shapes[3], np.float32)
        self._check(lib().les_get_aux(self.h, 0, _ptr(a), None, None))
        return a

    def get_rhs(self):
        a = np.zeros(self.shapes[3], np.float32)
        self._check(lib().les_get_aux(self.h, 1, _ptr(a), None, None))
        return a

    def _faces(self, which):
        su, sv, sw, _ = self.shapes
        a, b, c = np.zeros(su, np.float32), np.zeros(sv, np.float32), np.zeros(sw, np.float32)
        self._check(lib().les_get_aux(self.h, which, _ptr(a), _ptr(b), _ptr(c)))
        return a, b, c

    def get_force(self):
        return self._faces(2)

    def get_usum(self):
        return self._faces(3)

    def get_ghosted(self):
        s = (self.nz + 2, self.ny + 2, self.nx + 2)
        u, v, w = (np.zeros(s, np.float32) for _ in range(3))
        self._check(lib().les_get_ghosted(self.h, _ptr(u), _ptr(v), _ptr(w)))
        return u, v, w

    def get_timing(self, reset=True):
        """{kernel: (total ms, timed launches)} collected with params.timing = 1."""
        t = Timing()
        self._check(lib().les_get_timing(self.h, C.byref(t), int(bool(reset))))
        return {n: (t.ms[q], t.launches[q]) for q, n in enumerate(KERNEL_NAMES)}

    def autotune(self, reps=20):
        """Pick the fastest SOR sweep variant; returns (index, us per sweep per variant)."""
        ch = C.c_int32()
        us = np.zeros(NUM_SOR_VARIANTS, np.float64)
        self._check(lib().les_autotune(self.h, int(reps), C.byref(ch), _ptr(us)))
        return ch.value, us

    def set_sor_variant(self, v):
        return self._check(lib().les_set_sor_variant(self.h, int(v)))

    def get_step(self):
        s = C.c_int64()
        self._check(lib().les_get_step(self.h, C.byref(s)))
        return s.value

    def get_state(self) -> bytes:
        n = C.c_int64()
        self._check(lib().les_state_size(self.h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().les_get_state(self.h, buf, n))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        return self._check(lib().les_set_state(self.h, buf, len(blob)))



class Net:
    """The warm-start network (``lesnet_create``).  Device tensors are torch
    tensors (float32, contiguous, on the current device); work is ordered on
    torch's current stream."""

    def __init__(self, c1=16, c2=32, c3=64, seed=0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        cfg = NetConfig()
        lib().lesnet_default_config(C.byref(cfg))
        cfg.c1, cfg.c2, cfg.c3, cfg.seed = c1, c2, c3, seed
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        h = C.c_void_p()
        rc = lib().lesnet_create(C.byref(cfg), C.byref(h))
        if rc != LES_OK:
            raise LesError(rc, "lesnet_create failed")
        self.h = h
        self.channels = (c1, c2, c3)
        n = C.c_int64()
        lib().lesnet_num_params(self.h, C.byref(n))
        self.num_params = n.value

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.lesnet_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, rc):
        if rc != LES_OK:
            raise LesError(rc, lib().lesnet_last_error(self.h).decode())

    def get_params(self):
        out = np.zeros(self.num_params, np.float32)
        self._check(lib().lesnet_get_params(self.h, _ptr(out), self.num_params))
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32).reshape(-1)
        self._check(lib().lesnet_set_params(self.h, _ptr(a), a.size))

    def get_grads(self):
        out = np.zeros(self.num_params, np.float32)
        self._check(lib().lesnet_get_grads(self.h, _ptr(out), self.num_params))
        return out

    @staticmethod
    def _dims(x):
        if x.dim() != 5 or x.shape[4] != 3:
            raise ValueError("x must be [B, D, H, W, 3]")
        return tuple(int(d) for d in x.shape[:4])

    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def forward(self, x):
        import torch
        B, D, H, W = self._dims(x)
        y = torch.empty((B, D, H, W), dtype=torch.float32, device=x.device)
        self._check(lib().lesnet_forward(self.h, B, D, H, W, C.c_void_p(x.data_ptr()),
                                         C.c_void_p(y.data_ptr()), self._stream()))
        return y

    def gradients(self, x, dy):
        B, D, H, W = self._dims(x)
        self._check(lib().lesnet_gradients(self.h, B, D, H, W, C.c_void_p(x.data_ptr()),
                                           C.c_void_p(dy.data_ptr()), self._stream()))
        return self.get_grads()

    def set_lr(self, lr):
        self._check(lib().lesnet_set_lr(self.h, float(lr)))

    def train_step(self, x, t, want_loss=True):
        B, D, H, W = self._dims(x)
        loss = C.c_double(float("nan"))
        self._check(lib().lesnet_train_step(self.h, B, D, H, W, C.c_void_p(x.data_ptr()),
                                            C.c_void_p(t.data_ptr()),
                                            C.byref(loss) if want_loss else None, self._stream()))
        return loss.value


NET_OPS = {"conv3": 0, "conv3_dgrad": 1, "conv3_wgrad": 2, "up": 3, "up_dgrad": 4, "up_wgrad": 5}


def net_op(op: str, a, b, c=None, cin=None, cout=None):
    """One layer operation (``lesnet_op``) on torch device tensors; returns
    the float32 result as a torch tensor."""
    import torch

    code = NET_OPS[op]
    up = op.startswith("up")
    if op in ("conv3", "up"):
        B, D, H, W, cin = a.shape
        cout = b.shape[2]
        f = 2 if up else 1
        out = torch.empty((B, f * D, f * H, f * W, cout), device=a.device)
    elif op.endswith("dgrad"):
        B, D, H, W, cout = a.shape
        cin = b.shape[1]
        if up:
            D, H, W = D // 2, H // 2, W // 2
        out = torch.empty((B, D, H, W, cin), device=a.device)
    else:
        B, D, H, W, cin = a.shape
        cout = b.shape[4]
        out = torch.empty((8 if up else 27, cin, cout), device=a.device)
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    rc = lib().lesnet_op(code, B, D, H, W, cin, cout, ptr(a), ptr(b), ptr(c), ptr(out),
                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != LES_OK:
        raise LesError(rc, f"lesnet_op({op})")
    return out


def warm_grid(les: "LES"):
    D, H, W = C.c_int32(), C.c_int32(), C.c_int32()
    les._check(lib().les_warm_grid(les.h, C.byref(D), C.byref(H), C.byref(W)))
    return D.value, H.value, W.value


WARM_RESIDUAL, WARM_TRIAL, WARM_SMOOTH, WARM_ALWAYS = 0, 1, 2, 3


def set_warm_start(les: "LES", net: Optional[Net], target_scale: float = 1.0,
                   rule: int = WARM_RESIDUAL, param: int = 0, smooth: int = 0):
    """Warm-start the handle's solves with `net` (None: off); `rule`,
    `param` and `smooth` as in les_set_warm_start (lesnet.h)."""
    les._check(lib().les_set_warm_start(les.h, net.h if net is not None else None,
                                        float(target_scale), int(rule), int(param), int(smooth)))


def set_capture(les: "LES", d_x=None, d_t=None, smooth: int = 0):
    """Capture each step's network input / training target into the torch
    tensors d_x [D, H, W, 3] and d_t [D, H, W] (None, None: off), the
    target smoothed by `smooth` passes."""
    les._check(lib().les_set_capture(les.h, C.c_void_p(d_x.data_ptr()) if d_x is not None else None,
                                     C.c_void_p(d_t.data_ptr()) if d_t is not None else None,
                                     int(smooth)))


# ---- training-set preparation (lesnet.h): library kernels on torch memory


def _dev(t, what):
    if not (t.is_cuda and t.is_contiguous() and t.dtype.is_floating_point and t.element_size() == 4):
        raise ValueError(f"{what}: expected a contiguous float32 device tensor")
    return C.c_void_p(t.data_ptr())


def _net_check(rc, what):
    if rc != LES_OK:
        raise LesError(rc, what)


def crop(src, window, out=None, mirror_y: bool = False):
    """The window (z, y, x, cd, ch, cw) of src [D, H, W, C] or [D, H, W]
    into out [cd, ch, cw(, C)] (allocated if None), reflected in y with
    mirror_y (lesnet_crop)."""
    import torch
    z, y, x, cd, ch, cw = (int(v) for v in window)
    D, H, W = src.shape[:3]
    Cn = src.shape[3] if src.dim() == 4 else 1
    shape = (cd, ch, cw, Cn) if src.dim() == 4 else (cd, ch, cw)
    if out is None:
        out = torch.empty(shape, device=src.device, dtype=torch.float32)
    elif tuple(out.shape) != shape:
        raise ValueError(f"crop: out has shape {tuple(out.shape)}, expected {shape}")
    _net_check(lib().lesnet_crop(_dev(src, "crop"), D, H, W, Cn, z, y, x, cd, ch, cw, int(bool(mirror_y)),
                                 _dev(out, "crop"), C.c_void_p(_current_stream())), "lesnet_crop")
    return out


def gather(src, idx, out=None):
    """out[b] = src[idx[b]] along the first axis (lesnet_gather; at most 64
    items)."""
    import torch
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    n = int(idx.size)
    item = int(src[0].numel()) if src.shape[0] > 0 else 0
    if out is None:
        out = torch.empty((n,) + tuple(src.shape[1:]), device=src.device, dtype=torch.float32)
    _net_check(lib().lesnet_gather(_dev(src, "gather"), item, int(src.shape[0]),
                                   idx.ctypes.data_as(C.c_void_p), n, _dev(out, "gather"),
                                   C.c_void_p(_current_stream())), "lesnet_gather")
    return out


def sum_squares(x) -> float:
    """Sum of x^2 in float64, fixed-order (lesnet_sum_squares)."""
    import torch
    out = torch.empty(1, device=x.device, dtype=torch.float64)
    _net_check(lib().lesnet_sum_squares(_dev(x, "sum_squares"), int(x.numel()), C.c_void_p(out.data_ptr()),
                                        C.c_void_p(_current_stream())), "lesnet_sum_squares")
    return float(out.item())


def scale_div(x, s: float, out=None):
    """out = x / s elementwise in float32 (lesnet_scale_div)."""
    import torch
    if out is None:
        out = torch.empty_like(x)
    _net_check(lib().lesnet_scale_div(_dev(x, "scale_div"), int(x.numel()), float(s), _dev(out, "scale_div"),
                                      C.c_void_p(_current_stream())), "lesnet_scale_div")
    return out


def bc_range(nx: int, ny: int, nz: int) -> int:
    """Launch size of the boundary-range ghost refresh (les_bc_range)."""
    return int(lib().les_bc_range(C.byref(Grid(nx, ny, nz))))


def bc_map(nx: int, ny: int, nz: int, item: int):
    """(family, a, b) of a boundary-range item (les_bc_map)."""
    f, a, b = C.c_int32(), C.c_int32(), C.c_int32()
    rc = lib().les_bc_map(C.byref(Grid(nx, ny, nz)), int(item), C.byref(f), C.byref(a), C.byref(b))
    if rc != LES_OK:
        raise LesError(rc, "les_bc_map")
    return f.value, a.value, b.value


class Ensemble:
    """Several LES instances advanced together (les_ensemble_*).  Borrows the
    members: keep them alive and close the ensemble first."""

    def __init__(self, members):
        self.members = list(members)
        arr = (C.c_void_p * len(self.members))(*[m.h for m in self.members])
        h = C.c_void_p()
        rc = lib().les_ensemble_create(len(self.members), arr, C.byref(h))
        if rc != LES_OK:
            raise LesError(rc, "les_ensemble_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().les_ensemble_destroy(self.h)
            self.h = None

    __del__ = close

    def step(self, n=1):
        """Advance every member n steps: (status, stats, iterations[n, members])."""
        st = EnsembleStats()
        iters = np.zeros((max(int(n), 1), len(self.members)), np.int32)
        rc = lib().les_ensemble_step(self.h, int(n), C.byref(st), _ptr(iters))
        if rc not in (LES_OK, LES_NOT_CONVERGED):
            raise LesError(rc, lib().les_ensemble_last_error(self.h).decode())
        return rc, st.as_dict(), iters[:n].copy()

    def set_variant(self, variant):
        """Sweep variant of every member (-1: each member its own)."""
        rc = lib().les_ensemble_set_variant(self.h, int(variant))
        if rc != LES_OK:
            raise LesError(rc, "les_ensemble_set_variant")

    def set_mode(self, mode):
        rc = lib().les_ensemble_set_mode(self.h, int(mode))
        if rc != LES_OK:
            raise LesError(rc, "les_ensemble_set_mode")

    def autotune(self, reps=10):
        """Pick the fastest sweep variant for the whole ensemble:
        returns (index, us per half-sweep per variant)."""
        rc = lib().les_ensemble_autotune(self.h, int(reps))
        if rc != LES_OK:
            raise LesError(rc, lib().les_ensemble_last_error(self.h).decode())
        v = C.c_int32()
        us = np.zeros(NUM_SOR_VARIANTS, np.float64)
        lib().les_ensemble_tuning(self.h, C.byref(v), _ptr(us))
        return v.value, us
