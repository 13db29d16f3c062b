"""ctypes front end of the plain FP64 CPU oracle (hc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product package never imports it, and it
imports nothing from the product package.  See hc_oracle.c for what is computed
and which passage of the paper each piece follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hc_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

TOTAL_DEGREE = 0
LINEAR = 1

SUCCESS, AT_INFINITY, MIN_STEP, MAX_STEPS, SINGULAR, NONFINITE, REFINE_FAILED, SINGULAR_END = range(8)
STATUS_NAMES = ["SUCCESS", "AT_INFINITY", "MIN_STEP", "MAX_STEPS", "SINGULAR", "NONFINITE",
                "REFINE_FAILED", "SINGULAR_END"]


class Opts(ctypes.Structure):
    _fields_ = [
        ("h0", ctypes.c_double), ("h_min", ctypes.c_double), ("h_max", ctypes.c_double),
        ("beta_inc", ctypes.c_double), ("beta_dec", ctypes.c_double),
        ("tau", ctypes.c_double), ("pred_tol", ctypes.c_double), ("tau_refine", ctypes.c_double),
        ("inf_bound", ctypes.c_double), ("eta_max", ctypes.c_double),
        ("n_inc", ctypes.c_int), ("max_newton", ctypes.c_int),
        ("max_steps", ctypes.c_int), ("max_refine", ctypes.c_int),
    ]


# The paper prints no step-control constants (section 3 only says "a number of
# small steps"); these are the values both sides are run with.
DEFAULTS = dict(h0=0.05, h_min=1e-7, h_max=0.1, beta_inc=2.0, beta_dec=0.5, tau=1e-6,
                pred_tol=1e-2, tau_refine=1e-14, inf_bound=1e7, eta_max=1e-10, n_inc=5, max_newton=3,
                max_steps=5000, max_refine=10)


# Host threads at most: the CPU share a process gets beside one GPU on the
# machines this runs on (their nproc shows the whole host).
MAX_THREADS = 16


def default_threads() -> int:
    """Host threads the tracker uses by default: the cores this process may run
    on, at most MAX_THREADS."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, MAX_THREADS))


def default_opts(**kw) -> Opts:
    d = dict(DEFAULTS)
    d.update(kw)
    return Opts(**d)


class EgOpts(ctypes.Structure):
    """Power-series end-game options (orc_eg_opts in hc_oracle.c)."""
    _fields_ = [("s0", ctypes.c_double), ("beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("tol_inf", ctypes.c_double),
                ("tau", ctypes.c_double), ("h_min", ctypes.c_double), ("max_newton", ctypes.c_int),
                ("max_samples", ctypes.c_int),
                ("max_cycle", ctypes.c_int), ("every", ctypes.c_int)]


# The end-game's constants (ours: the paper has no end-game).
EG_DEFAULTS = dict(s0=0.1, beta=0.25, tol=1e-9, tol_inf=1e-3, tau=1e-8, h_min=1e-14, max_newton=5, max_samples=16,
                   max_cycle=8, every=0)


def default_eg_opts(**kw) -> EgOpts:
    d = dict(EG_DEFAULTS)
    d.update(kw)
    return EgOpts(**d)


class _System(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_terms", ctypes.c_int),
                ("term_eq", ctypes.POINTER(ctypes.c_int)),
                ("term_exp", ctypes.POINTER(ctypes.c_int))]


INFO_DTYPE = np.dtype([("steps", np.int32), ("rejects", np.int32), ("newton_its", np.int32),
                       ("refine_its", np.int32), ("residual", np.float64)], align=True)


def build(force: bool = False) -> str:
    """Compile hc_oracle.c into liborc.so next to it (plain gcc, -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


# The CPU baseline's build of the same source: tuned for the host it runs on.
# Auto-vectorisation stays off: gcc 11's AVX-512 code for the LU's row swap
# assumes 32-byte alignment of rows that are 16 bytes apart and faults, and the
# scalar complex arithmetic gains nothing from it (measured on the CPU).
NATIVE_FLAGS = "-O3 -march=native -fno-tree-vectorize"
_NATIVE_LIB = os.path.join(_HERE, "liborc_native.so")


def build_native() -> str:
    """Compile hc_oracle.c with NATIVE_FLAGS into liborc_native.so (on the host
    that will run it: -march=native)."""
    tmp = _NATIVE_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *NATIVE_FLAGS.split(), "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                           "-lm", "-lpthread"])
    os.replace(tmp, _NATIVE_LIB)
    return _NATIVE_LIB


def use_native_build() -> str:
    """Switch this process's oracle to the NATIVE_FLAGS build; returns its path."""
    global _lib, _lib_path
    path = build_native()
    _lib = None
    _lib_path = path
    _load()
    return path


_lib = None
_lib_path = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_lib_path or build())
        P = ctypes.c_void_p
        lib.orc_track_batch.restype = ctypes.c_int
        lib.orc_track_batch.argtypes = [ctypes.POINTER(_System), ctypes.c_int, P, P, P, P,
                                        ctypes.c_int, ctypes.c_int, ctypes.POINTER(Opts),
                                        ctypes.c_int, P, P, P]
        lib.orc_track_batch_eg.restype = ctypes.c_int
        lib.orc_track_batch_eg.argtypes = [ctypes.POINTER(_System), ctypes.c_int, P, P, P, P,
                                           ctypes.c_int, ctypes.c_int, ctypes.POINTER(Opts),
                                           ctypes.POINTER(EgOpts), ctypes.c_int, P, P, P, P]
        lib.orc_eg_extrapolate.restype = ctypes.c_int
        lib.orc_eg_extrapolate.argtypes = [ctypes.c_int, P, P, P, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int), P]
        lib.orc_eval_system.restype = None
        lib.orc_eval_system.argtypes = [ctypes.POINTER(_System), P, P, P, P]
        lib.orc_homotopy_eval_flat.restype = None
        lib.orc_homotopy_eval_flat.argtypes = [ctypes.POINTER(_System), ctypes.c_int, P, P,
                                               ctypes.c_double, ctypes.c_double, P,
                                               ctypes.c_double, P, P, P]
        lib.orc_lu_solve.restype = ctypes.c_int
        lib.orc_lu_solve.argtypes = [ctypes.c_int, P, P, P]
        lib.orc_rk4_fixed.restype = ctypes.c_int
        lib.orc_rk4_fixed.argtypes = [ctypes.POINTER(_System), ctypes.c_int, P, P,
                                      ctypes.c_double, ctypes.c_double, P, ctypes.c_int, P]
        lib.orc_newton_trace.restype = ctypes.c_int
        lib.orc_newton_trace.argtypes = [ctypes.POINTER(_System), ctypes.c_int, P, P,
                                         ctypes.c_double, ctypes.c_double, P, ctypes.c_double,
                                         ctypes.c_int, P, P]
        lib.orc_residual.restype = ctypes.c_double
        lib.orc_residual.argtypes = [ctypes.POINTER(_System), P, P]
        lib.orc_degrees.restype = None
        lib.orc_degrees.argtypes = [ctypes.POINTER(_System), P]
        lib.orc_total_degree_start.restype = None
        lib.orc_total_degree_start.argtypes = [ctypes.c_int, P, ctypes.c_longlong, P]
        _lib = lib
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Sys:
    """Keeps the int32 arrays alive while the C struct points at them."""

    def __init__(self, system):
        self.term_eq = np.ascontiguousarray(system.term_eq, dtype=np.int32)
        self.term_exp = np.ascontiguousarray(system.term_exp, dtype=np.int32)
        self.n = int(system.n)
        self.c = _System(self.n, int(self.term_eq.shape[0]),
                         self.term_eq.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                         self.term_exp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))


def degrees(system) -> np.ndarray:
    s = _Sys(system)
    d = np.zeros(s.n, np.int32)
    _load().orc_degrees(ctypes.byref(s.c), _ptr(d))
    return d


def total_degree_start(system, b: int) -> np.ndarray:
    d = degrees(system)
    x = np.zeros(len(d), np.complex128)
    _load().orc_total_degree_start(len(d), _ptr(d), int(b), _ptr(x))
    return x


def eval_system(system, coef, x):
    """(F [n], J [n, n]) at x."""
    s = _Sys(system)
    c, xx = _c128(coef), _c128(x)
    F = np.zeros(s.n, np.complex128)
    J = np.zeros((s.n, s.n), np.complex128)
    _load().orc_eval_system(ctypes.byref(s.c), _ptr(c), _ptr(xx), _ptr(F), _ptr(J))
    return F, J


def homotopy_eval(system, x, t, coef1, gamma=1.0, coef0=None, kind=TOTAL_DEGREE):
    """(H [n], H_x [n, n], H_t [n]) at (x, t)."""
    s = _Sys(system)
    c1 = _c128(coef1)
    c0 = None if coef0 is None else _c128(coef0)
    xx = _c128(x)
    H = np.zeros(s.n, np.complex128)
    Hx = np.zeros((s.n, s.n), np.complex128)
    Ht = np.zeros(s.n, np.complex128)
    g = complex(gamma)
    _load().orc_homotopy_eval_flat(ctypes.byref(s.c), kind, _ptr(c0), _ptr(c1), g.real, g.imag,
                                   _ptr(xx), float(t), _ptr(H), _ptr(Hx), _ptr(Ht))
    return H, Hx, Ht


def lu_solve(A, b):
    """x with A x = b, or None if a pivot is exactly zero."""
    A = _c128(A)
    b = _c128(b)
    n = b.shape[0]
    x = np.zeros(n, np.complex128)
    if _load().orc_lu_solve(n, _ptr(A), _ptr(b), _ptr(x)):
        return None
    return x


def rk4_fixed(system, x0, n_steps, coef1, gamma=1.0, coef0=None, kind=TOTAL_DEGREE):
    s = _Sys(system)
    c1 = _c128(coef1)
    c0 = None if coef0 is None else _c128(coef0)
    x = _c128(x0)
    out = np.zeros(s.n, np.complex128)
    g = complex(gamma)
    if _load().orc_rk4_fixed(ctypes.byref(s.c), kind, _ptr(c0), _ptr(c1), g.real, g.imag,
                             _ptr(x), int(n_steps), _ptr(out)):
        return None
    return out


def newton_trace(system, x0, t, iters, coef1, gamma=1.0, coef0=None, kind=TOTAL_DEGREE):
    s = _Sys(system)
    c1 = _c128(coef1)
    c0 = None if coef0 is None else _c128(coef0)
    x = _c128(x0)
    out = np.zeros(s.n, np.complex128)
    norms = np.zeros(iters, np.float64)
    g = complex(gamma)
    if _load().orc_newton_trace(ctypes.byref(s.c), kind, _ptr(c0), _ptr(c1), g.real, g.imag,
                                _ptr(x), float(t), int(iters), _ptr(norms), _ptr(out)):
        return None, None
    return norms, out


def eg_extrapolate(y0, y1, y2, beta, max_cycle=8):
    """The end-game's estimator: (cycle number, extrapolated vector) from samples
    at s, beta s, beta^2 s, or None if they do not decay."""
    a, b, c = _c128(y0), _c128(y1), _c128(y2)
    E = np.zeros_like(a)
    cyc = ctypes.c_int(0)
    if _load().orc_eg_extrapolate(len(a), _ptr(a), _ptr(b), _ptr(c), float(beta), int(max_cycle),
                                  ctypes.byref(cyc), _ptr(E)):
        return None
    return cyc.value, E


def residual(system, coef, x) -> float:
    s = _Sys(system)
    c, xx = _c128(coef), _c128(x)
    return float(_load().orc_residual(ctypes.byref(s.c), _ptr(c), _ptr(xx)))


def track(system, coef1, gamma=None, start=None, coef0=None, kind=TOTAL_DEGREE, opts=None,
          n_threads: Optional[int] = None, endgame=None):
    """Track every start point for every instance.

    coef1: [n_inst, n_terms] target coefficients; gamma: [n_inst] (total degree);
    start: [n_start, n] start points or None for the total-degree start points;
    coef0: [n_terms] start coefficients (LINEAR); endgame: None, True (the
    default end-game options) or an EgOpts.
    Returns endpoints [n_inst, n_start, n], status [n_inst, n_start] (int32),
    info [n_inst, n_start] (INFO_DTYPE); with an end-game also the cycle numbers
    [n_inst, n_start] (int32, 0 where no end-game converged).
    """
    s = _Sys(system)
    c1 = _c128(coef1)
    if c1.ndim == 1:
        c1 = c1[None, :]
    n_inst = c1.shape[0]
    g = None if gamma is None else _c128(np.broadcast_to(np.asarray(gamma), (n_inst,)))
    if start is None:
        if kind != TOTAL_DEGREE:
            raise ValueError("a parameter homotopy needs start points")
        n_start = int(np.prod(degrees(system).astype(np.int64)))
        st = None
    else:
        st = _c128(start).reshape(-1, s.n)
        n_start = st.shape[0]
    c0 = None if coef0 is None else _c128(coef0)
    ep = np.zeros((n_inst, n_start, s.n), np.complex128)
    status = np.zeros((n_inst, n_start), np.int32)
    info = np.zeros((n_inst, n_start), INFO_DTYPE)
    o = opts if opts is not None else default_opts()
    nt = n_threads if n_threads is not None else default_threads()
    if endgame is None or endgame is False:
        rc = _load().orc_track_batch(ctypes.byref(s.c), kind, _ptr(c0), _ptr(c1), _ptr(g), _ptr(st),
                                     n_start, n_inst, ctypes.byref(o), int(nt), _ptr(ep),
                                     _ptr(status), _ptr(info))
        if rc != 0:
            raise ValueError("orc_track_batch rejected its arguments")
        return ep, status, info
    eg = default_eg_opts() if endgame is True else endgame
    cyc = np.zeros((n_inst, n_start), np.int32)
    rc = _load().orc_track_batch_eg(ctypes.byref(s.c), kind, _ptr(c0), _ptr(c1), _ptr(g), _ptr(st),
                                    n_start, n_inst, ctypes.byref(o), ctypes.byref(eg), int(nt), _ptr(ep),
                                    _ptr(status), _ptr(info), _ptr(cyc))
    if rc != 0:
        raise ValueError("orc_track_batch_eg rejected its arguments")
    return ep, status, info, cyc
