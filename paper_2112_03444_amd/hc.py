"""Thin ctypes binding of libhc.so (include/hc.h).

Argument marshalling only: every step of the tracking runs in the library's HIP
kernels.  If libhc.so is missing the import of the binding fails loudly; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import contextlib

import numpy as np

_nullcontext = contextlib.nullcontext

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhc.so")

HC_OK = 0
HC_TOTAL_DEGREE, HC_PARAMETER = 0, 1
HC_FP64, HC_MIXED = 0, 1
(HC_T_SUCCESS, HC_T_AT_INFINITY, HC_T_MIN_STEP, HC_T_MAX_STEPS, HC_T_SINGULAR, HC_T_NONFINITE,
 HC_T_REFINE_FAILED, HC_T_SINGULAR_END) = range(8)
STATUS_NAMES = ["SUCCESS", "AT_INFINITY", "MIN_STEP", "MAX_STEPS", "SINGULAR", "NONFINITE",
                "REFINE_FAILED", "SINGULAR_END"]
HC_MAX_N = 32
HC_NOALLOC_SCRATCH_BYTES = 64 << 20  # fixed workspace of hc_track_device_noalloc, per device
HC_LAYOUT_AUTO, HC_LAYOUT_DENSE, HC_LAYOUT_TERMS = 0, 1, 2
HC_EVAL_ROWS, HC_EVAL_MFMA = 0, 1


class HcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hc error {code}: {msg}")
        self.code = code


class SystemDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("term_eq", ctypes.c_void_p), ("term_exp", ctypes.c_void_p),
                ("n_params", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("coef_const", ctypes.c_void_p), ("coef_rowptr", ctypes.c_void_p),
                ("coef_col", ctypes.c_void_p), ("coef_val", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("h0", "h_min", "h_max", "beta_inc", "beta_dec", "tau64", "tau32", "pred_tol",
                 "tau_refine", "inf_bound", "eta_max", "t_end")] + \
               [(k, ctypes.c_int32) for k in
                ("precision", "n_inc", "max_newton", "max_steps", "max_refine",
                 "steps_per_launch", "tracks_per_item", "lanes_per_path", "use_graph", "fp64_residual",
                 "crossing_check", "per_instance_start", "table_layout", "endgame", "eg_max_newton",
                 "eg_max_samples", "eg_max_cycle")] + \
               [(k, ctypes.c_double) for k in
                ("eg_s0", "eg_beta", "eg_tol", "eg_tol_inf", "eg_tau", "eg_h_min")]


class Job(ctypes.Structure):
    _fields_ = [("sys", ctypes.c_void_p), ("start", ctypes.c_void_p), ("n_start", ctypes.c_int32),
                ("n_inst", ctypes.c_int32), ("p_start", ctypes.c_void_p), ("p_target", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p), ("endpoints", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("info", ctypes.c_void_p)]


class Profile(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in
                ("ms_prep", "ms_init", "ms_track_fp32", "ms_track_fp64", "ms_refine")] + \
               [("launches_fp32", ctypes.c_int32), ("launches_fp64", ctypes.c_int32),
                ("ms_crossing", ctypes.c_float), ("stages_fp32", ctypes.c_int64),
                ("stages_fp64", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


INFO_DTYPE = np.dtype([("steps", np.int32), ("rejects", np.int32), ("newton_its", np.int32),
                       ("refine_its", np.int32), ("escalated", np.int32), ("cycle", np.int32),
                       ("residual", np.float64)])
assert INFO_DTYPE.itemsize == 32

_lib = None


def lib():
    """The loaded libhc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch-ROCm ships its own HIP runtime with the same soname as the system
        # one.  Loading torch first lets libhc bind to that already-loaded runtime,
        # so the process holds a single HIP runtime shared with torch's allocator.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2112_03444_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.hc_default_opts.restype = None
        L.hc_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.hc_last_error.restype = ctypes.c_char_p
        L.hc_last_error.argtypes = []
        L.hc_create.restype = ctypes.c_int
        L.hc_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
        L.hc_destroy.restype = None
        L.hc_destroy.argtypes = [P]
        L.hc_load_system.restype = ctypes.c_int
        L.hc_load_system.argtypes = [P, ctypes.POINTER(SystemDesc), ctypes.POINTER(P)]
        L.hc_load_system_layout.restype = ctypes.c_int
        L.hc_load_system_layout.argtypes = [P, ctypes.POINTER(SystemDesc), I32, ctypes.POINTER(P)]
        L.hc_free_system.restype = ctypes.c_int
        L.hc_free_system.argtypes = [P, P]
        L.hc_system_dims.restype = ctypes.c_int
        L.hc_system_dims.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]
        L.hc_total_degree_start.restype = ctypes.c_int
        L.hc_total_degree_start.argtypes = [P, I64, I64, P]
        L.hc_track.restype = ctypes.c_int
        L.hc_track.argtypes = [P, P, P, I32, P, P, I32, P, ctypes.POINTER(Opts), P, P, P]
        L.hc_track_device.restype = ctypes.c_int
        L.hc_track_device.argtypes = [P, P, P, I32, P, P, I32, P, ctypes.POINTER(Opts), P, P, P, P]
        L.hc_track_device_noalloc.restype = ctypes.c_int
        L.hc_track_device_noalloc.argtypes = [P, P, P, I32, P, P, I32, P, ctypes.POINTER(Opts), P, P, P, P]
        L.hc_tune_save.restype = ctypes.c_int
        L.hc_tune_save.argtypes = [P, ctypes.c_char_p]
        L.hc_tune_load.restype = ctypes.c_int
        L.hc_tune_load.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I32)]
        L.hc_autotune.restype = ctypes.c_int
        L.hc_autotune.argtypes = [P, P, P, I32, P, P, I32, P, ctypes.POINTER(Opts), P, P, P, P,
                                  ctypes.POINTER(Opts)]
        L.hc_track_batch_device.restype = ctypes.c_int
        L.hc_track_batch_device.argtypes = [P, I32, ctypes.POINTER(Job), ctypes.POINTER(Opts), P]
        L.hc_set_profiling.restype = ctypes.c_int
        L.hc_set_profiling.argtypes = [P, I32]
        L.hc_last_profile.restype = ctypes.c_int
        L.hc_last_profile.argtypes = [P, ctypes.POINTER(Profile)]
        L.hc_solve_batched_device.restype = ctypes.c_int
        L.hc_solve_batched_device.argtypes = [P, I32, I64, I32, P, P, P, P, P]
        L.hc_measure_vector_peak.restype = ctypes.c_int
        L.hc_measure_vector_peak.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double)]
        L.hc_distinct_device.restype = ctypes.c_int
        L.hc_distinct_device.argtypes = [P, I32, I64, P, ctypes.c_double, P, P]
        L.hc_eval_dense_device.restype = ctypes.c_int
        L.hc_eval_dense_device.argtypes = [P, P, P, I32, P, I32, I32, I32, P, P, P]
        L.hc_homogenize.restype = ctypes.c_int
        L.hc_homogenize.argtypes = [I32, I32, P, P, P, P, I32, I32, P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != HC_OK:
        raise HcError(rc, lib().hc_last_error().decode())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().hc_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": HC_FP64, "mixed": HC_MIXED}[v]
        setattr(o, k, v)
    return o


def homogenize(n: int, entries, K: int, M: int) -> np.ndarray:
    """Section-6 term tables.  entries: list of polynomials, each a list of
    (scalar, coef_index, exponent_vector).  Returns int32 [n_entries, K, 2 + M]."""
    ptr = [0]
    sc, cf, ex = [], [], []
    for e in entries:
        for (s, a, expv) in e:
            sc.append(int(s))
            cf.append(int(a))
            ex.append(np.asarray(expv, np.int32))
        ptr.append(len(sc))
    ptr_a = np.asarray(ptr, np.int32)
    sc_a = np.asarray(sc, np.int32)
    cf_a = np.asarray(cf, np.int32)
    ex_a = np.ascontiguousarray(np.stack(ex) if ex else np.zeros((0, n), np.int32), dtype=np.int32)
    out = np.zeros((len(entries), K, 2 + M), np.int32)
    _check(lib().hc_homogenize(n, len(entries), _ptr(ptr_a), _ptr(sc_a), _ptr(cf_a), _ptr(ex_a),
                               K, M, _ptr(out)))
    return out


class System:
    def __init__(self, ctx: "Context", handle: ctypes.c_void_p):
        self.ctx = ctx
        self.handle = handle
        n = ctypes.c_int32()
        b = ctypes.c_int64()
        _check(lib().hc_system_dims(handle, ctypes.byref(n), ctypes.byref(b)))
        self.n = n.value
        self.bezout = b.value

    def total_degree_start(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = self.bezout - first
        out = np.zeros((count, self.n), np.complex128)
        _check(lib().hc_total_degree_start(self.handle, first, count, _ptr(out)))
        return out


class Context:
    """One hc_ctx on HIP device `device`."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hc_create(device, ctypes.byref(h)))
        self.handle = h
        self._systems = []

    def close(self):
        if self.handle:
            lib().hc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_system(self, system, kind: int = HC_TOTAL_DEGREE, coef_const=None, coef_map=None,
                    layout: int = HC_LAYOUT_AUTO) -> System:
        """system: object with n, term_eq [n_terms], term_exp [n_terms, n].
        coef_map: None (identity, p = coefficients) or (rowptr, col, val) CSR.
        layout: HC_LAYOUT_AUTO, HC_LAYOUT_DENSE or HC_LAYOUT_TERMS."""
        te = np.ascontiguousarray(system.term_eq, np.int32)
        tx = np.ascontiguousarray(system.term_exp, np.int32)
        keep = [te, tx]
        d = SystemDesc()
        d.n = int(system.n)
        d.n_terms = int(te.shape[0])
        d.term_eq = te.ctypes.data
        d.term_exp = tx.ctypes.data
        d.kind = kind
        if coef_const is not None:
            cc = np.ascontiguousarray(coef_const, np.complex128)
            keep.append(cc)
            d.coef_const = cc.ctypes.data
        if coef_map is None:
            d.n_params = d.n_terms
        else:
            rp, col, val, n_params = coef_map
            rp = np.ascontiguousarray(rp, np.int32)
            col = np.ascontiguousarray(col, np.int32)
            val = np.ascontiguousarray(val, np.complex128)
            keep += [rp, col, val]
            d.n_params = int(n_params)
            d.coef_rowptr = rp.ctypes.data
            d.coef_col = col.ctypes.data if col.size else None
            d.coef_val = val.ctypes.data if val.size else None
        h = ctypes.c_void_p()
        _check(lib().hc_load_system_layout(self.handle, ctypes.byref(d), int(layout), ctypes.byref(h)))
        del keep
        s = System(self, h)
        self._systems.append(s)
        return s

    def set_profiling(self, enable: bool = True):
        _check(lib().hc_set_profiling(self.handle, 1 if enable else 0))

    def last_profile(self) -> Profile:
        p = Profile()
        _check(lib().hc_last_profile(self.handle, ctypes.byref(p)))
        return p

    def free_system(self, s: System):
        _check(lib().hc_free_system(self.handle, s.handle))
        self._systems.remove(s)

    def track(self, s: System, p_target, gamma=None, start=None, p_start=None, opts: Optional[Opts] = None,
              n_start: Optional[int] = None):
        """Host-buffer hc_track.  p_target [n_inst, n_params]; gamma [n_inst];
        start [n_start, n] or None (total-degree points).  A start of shape
        [n_inst, n_start, n] or a p_start of shape [n_inst, n_params] gives every
        instance its own start system (opts.per_instance_start; the other one is
        broadcast).  Returns numpy (endpoints [n_inst, n_start, n],
        status [n_inst, n_start], info)."""
        p = np.ascontiguousarray(p_target, np.complex128)
        if p.ndim == 1:
            p = p[None, :]
        n_inst = p.shape[0]
        g = None if gamma is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(gamma, np.complex128), (n_inst,)))
        st = None if start is None else np.asarray(start, np.complex128)
        ps = None if p_start is None else np.asarray(p_start, np.complex128)
        per_inst = (st is not None and st.ndim == 3) or (ps is not None and ps.ndim == 2)
        if per_inst:
            if st is not None:
                st = st if st.ndim == 3 else np.broadcast_to(st.reshape(-1, s.n), (n_inst,) + st.reshape(-1, s.n).shape)
                if st.shape[0] != n_inst:
                    raise ValueError("start must hold one set of start points per instance")
            if ps is not None:
                ps = ps if ps.ndim == 2 else np.broadcast_to(ps, (n_inst, ps.shape[0]))
                if ps.shape[0] != n_inst:
                    raise ValueError("p_start must hold one parameter vector per instance")
        if st is not None:
            if n_start is None:
                n_start = st.shape[1] if per_inst else st.reshape(-1, s.n).shape[0]
            st = np.ascontiguousarray(st).reshape(-1, s.n)
        if n_start is None:
            n_start = s.bezout
        ps = None if ps is None else np.ascontiguousarray(ps)
        ep = np.zeros((n_inst, n_start, s.n), np.complex128)
        status = np.zeros((n_inst, n_start), np.int32)
        info = np.zeros((n_inst, n_start), INFO_DTYPE)
        o = opts if opts is not None else default_opts()
        if per_inst:
            o = Opts.from_buffer_copy(o)
            o.per_instance_start = 1
        _check(lib().hc_track(self.handle, s.handle, _ptr(st), n_start, _ptr(ps), _ptr(p), n_inst, _ptr(g),
                              ctypes.byref(o), _ptr(ep), _ptr(status), _ptr(info)))
        return ep, status, info

    def track_device(self, s: System, p_target, gamma, endpoints, status, info=None, start=None,
                     p_start=None, n_start: Optional[int] = None, opts: Optional[Opts] = None, stream=None,
                     noalloc: bool = False):
        """Device-pointer hc_track_device on torch tensors (complex128 for complex
        arrays, int32 status, info as a [.., 32]-byte uint8 tensor or None).
        `stream` is a torch.cuda.Stream (default: the current stream).  With
        noalloc the call goes to hc_track_device_noalloc (the library's fixed
        device workspace, no allocation)."""
        import torch

        def dp(t):
            return None if t is None else ctypes.c_void_p(t.data_ptr())

        n_inst = p_target.shape[0]
        per_inst = (start is not None and start.dim() == 3) or (p_start is not None and p_start.dim() == 2)
        if n_start is None:
            n_start = s.bezout if start is None else start.shape[1 if start.dim() == 3 else 0]
        if stream is None:
            stream = torch.cuda.current_stream()
        o = opts if opts is not None else default_opts()
        if per_inst:
            # both start arrays must then be per instance
            if (start is not None and start.dim() != 3) or (p_start is not None and p_start.dim() != 2):
                raise ValueError("per-instance start: start [n_inst, n_start, n] and p_start [n_inst, n_params]")
            o = Opts.from_buffer_copy(o)
            o.per_instance_start = 1
        fn = lib().hc_track_device_noalloc if noalloc else lib().hc_track_device
        _check(fn(self.handle, s.handle, dp(start), n_start, dp(p_start), dp(p_target), n_inst, dp(gamma),
                  ctypes.byref(o), dp(endpoints), dp(status), dp(info), ctypes.c_void_p(stream.cuda_stream)))

    def autotune(self, s: System, p_target, gamma, endpoints, status, info=None, start=None, p_start=None,
                 n_start: Optional[int] = None, opts: Optional[Opts] = None, stream=None) -> Opts:
        """hc_autotune on torch tensors; returns the chosen options."""
        import torch

        def dp(t):
            return None if t is None else ctypes.c_void_p(t.data_ptr())

        n_inst = p_target.shape[0]
        if n_start is None:
            n_start = s.bezout if start is None else start.shape[0]
        if stream is None:
            stream = torch.cuda.current_stream()
        o = opts if opts is not None else default_opts()
        best = Opts()
        _check(lib().hc_autotune(self.handle, s.handle, dp(start), n_start, dp(p_start), dp(p_target), n_inst,
                                 dp(gamma), ctypes.byref(o), dp(endpoints), dp(status), dp(info),
                                 ctypes.c_void_p(stream.cuda_stream), ctypes.byref(best)))
        return best

    def tune_save(self, path: str):
        """hc_tune_save: the autotuner's choices to a text file."""
        _check(lib().hc_tune_save(self.handle, os.fsencode(path)))

    def tune_load(self, path: str) -> int:
        """hc_tune_load: merge stored autotuner choices; returns the entry count."""
        n = ctypes.c_int32()
        _check(lib().hc_tune_load(self.handle, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def track_piecewise(self, s: System, waypoints, start, opts: Optional[Opts] = None):
        """Parameter homotopy along a piecewise-linear path of coefficient
        vectors: waypoints[0] [n_params] (shared start instance), then
        waypoints[1..L] each [n_inst, n_params]; leg l is one hc_track call from
        waypoints[l-1] to waypoints[l], started at the previous leg's endpoints
        (per instance from leg 2 on; a path that failed is started at NaN, so it
        ends at once as non-finite).  Returns the last leg's (endpoints, status,
        info)."""
        pts = np.ascontiguousarray(start, np.complex128)
        c_prev = np.asarray(waypoints[0], np.complex128)
        ep = st = info = None
        for c_next in waypoints[1:]:
            ep, st, info = self.track(s, c_next, start=pts, p_start=c_prev, opts=opts)
            pts = np.where((st == HC_T_SUCCESS)[..., None], ep, np.nan + 0j)
            c_prev = np.asarray(c_next, np.complex128)
        return ep, st, info

    def track_piecewise_device(self, s: System, waypoints, start, endpoints, status, info=None,
                               opts: Optional[Opts] = None, stream=None):
        """track_piecewise on device tensors: waypoints as torch complex128
        tensors ([n_params], then [n_inst, n_params] each), start [n_start, n];
        endpoints/status/info receive the last leg's results.  The legs run on
        `stream` back to back (no host synchronisation)."""
        import torch
        n_inst = waypoints[1].shape[0]
        pts = start
        c_prev = waypoints[0]
        for li, c_next in enumerate(waypoints[1:]):
            self.track_device(s, c_next, None, endpoints, status, info, start=pts, p_start=c_prev, opts=opts,
                              stream=stream)
            if li + 2 < len(waypoints):
                with torch.cuda.stream(stream) if stream is not None else _nullcontext():
                    pts = torch.where((status == HC_T_SUCCESS)[..., None], endpoints,
                                      torch.full_like(endpoints, complex(float("nan"), 0.0)))
                c_prev = c_next
                if c_prev.dim() == 1:
                    c_prev = c_prev.expand(n_inst, -1).contiguous()
        return endpoints, status, info

    def solve_batched_device(self, A, b, x, info=None, stream=None):
        """hc_solve_batched_device on torch tensors: A [batch, n, n], b and x
        [batch, n], all complex64 (FP32) or all complex128 (FP64), contiguous, on
        the context's device; info [batch] int32 or None.  Enqueued on `stream`
        (default: the current stream)."""
        import torch
        batch, n = A.shape[0], A.shape[1]
        if A.shape != (batch, n, n) or b.shape != (batch, n) or x.shape != (batch, n):
            raise ValueError("shapes: A [batch, n, n], b and x [batch, n]")
        if not (A.dtype == b.dtype == x.dtype) or A.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("A, b, x must all be complex64 or all complex128")
        if not (A.is_contiguous() and b.is_contiguous() and x.is_contiguous()):
            raise ValueError("A, b, x must be contiguous")
        if info is not None and (info.dtype != torch.int32 or info.shape != (batch,)):
            raise ValueError("info must be int32 [batch]")
        if stream is None:
            stream = torch.cuda.current_stream()
        fp32 = 1 if A.dtype == torch.complex64 else 0
        _check(lib().hc_solve_batched_device(self.handle, n, batch, fp32, ctypes.c_void_p(A.data_ptr()),
                                             ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                             None if info is None else ctypes.c_void_p(info.data_ptr()),
                                             ctypes.c_void_p(stream.cuda_stream)))

    def distinct_device(self, points, tol: float = 1e-8, stream=None):
        """hc_distinct_device on a complex128 torch tensor [count, n]: the int32
        keep mask (1 = no earlier point within tol)."""
        import torch
        pts = points.contiguous()
        keep = torch.empty(pts.shape[0], dtype=torch.int32, device=pts.device)
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().hc_distinct_device(self.handle, pts.shape[1], pts.shape[0], ctypes.c_void_p(pts.data_ptr()),
                                        float(tol), ctypes.c_void_p(keep.data_ptr()),
                                        ctypes.c_void_p(stream.cuda_stream)))
        return keep

    def eval_dense_device(self, sys: "System", p_target, x, engine: int = 0, repeat: int = 1, F=None, J=None,
                          stream=None):
        """hc_eval_dense_device: F and its Jacobian in FP32 at the points x
        (complex64 [n_inst, n_pts, n] on the device) of the instances whose
        coefficients (parameters) are p_target (complex128 [n_inst, n_params]).
        engine: HC_EVAL_ROWS (0, vector ALUs) or HC_EVAL_MFMA (1, matrix cores).
        Returns (F [n_inst, n_pts, n], J [n_inst, n_pts, n, n]), complex64."""
        import torch
        if x.dim() != 3 or x.dtype != torch.complex64 or not x.is_contiguous():
            raise ValueError("x must be a contiguous complex64 tensor [n_inst, n_pts, n]")
        n_inst, n_pts, n = x.shape
        if n != sys.n:
            raise ValueError(f"x has {n} unknowns, the system {sys.n}")
        p = p_target.contiguous()
        if p.dtype != torch.complex128 or p.shape[0] != n_inst:
            raise ValueError("p_target must be complex128 [n_inst, n_params]")
        if F is None:
            F = torch.empty((n_inst, n_pts, n), dtype=torch.complex64, device=x.device)
        if J is None:
            J = torch.empty((n_inst, n_pts, n, n), dtype=torch.complex64, device=x.device)
        if F.shape != (n_inst, n_pts, n) or J.shape != (n_inst, n_pts, n, n):
            raise ValueError("F must be [n_inst, n_pts, n] and J [n_inst, n_pts, n, n]")
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(lib().hc_eval_dense_device(self.handle, sys.handle, ctypes.c_void_p(p.data_ptr()), n_inst,
                                          ctypes.c_void_p(x.data_ptr()), n_pts, int(engine), int(repeat),
                                          ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(J.data_ptr()),
                                          ctypes.c_void_p(stream.cuda_stream)))
        return F, J

    def measure_vector_peak(self, fp64: bool) -> float:
        """hc_measure_vector_peak: the device's measured FMA rate in TFLOP/s
        (FP64, or plain one-value-per-lane FP32)."""
        v = ctypes.c_double(0.0)
        _check(lib().hc_measure_vector_peak(self.handle, 1 if fp64 else 0, ctypes.byref(v)))
        return v.value

    def track_batch_device(self, jobs, opts: Optional[Opts] = None, stream=None):
        """hc_track_batch_device.  jobs: list of dicts with keys sys (System),
        p_target, endpoints, status and optionally gamma, info, start, p_start,
        n_start (torch tensors on the device, as in track_device)."""
        import torch

        def dp(t):
            return None if t is None else t.data_ptr()

        arr = (Job * max(len(jobs), 1))()
        for k, j in enumerate(jobs):
            s = j["sys"]
            start = j.get("start")
            n_start = j.get("n_start")
            if n_start is None:
                n_start = s.bezout if start is None else start.shape[0]
            arr[k] = Job(s.handle.value if hasattr(s.handle, "value") else s.handle, dp(start), n_start,
                         j["p_target"].shape[0], dp(j.get("p_start")), dp(j["p_target"]), dp(j.get("gamma")),
                         dp(j["endpoints"]), dp(j["status"]), dp(j.get("info")))
        if stream is None:
            stream = torch.cuda.current_stream()
        o = opts if opts is not None else default_opts()
        _check(lib().hc_track_batch_device(self.handle, len(jobs), arr, ctypes.byref(o),
                                           ctypes.c_void_p(stream.cuda_stream)))


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("max_batch_requests", ctypes.c_int32),
                ("hbm_budget", ctypes.c_int64), ("opts", Opts)]


class Request(ctypes.Structure):
    _fields_ = [("sys", ctypes.c_void_p), ("n_start", ctypes.c_int32), ("n_inst", ctypes.c_int32),
                ("start", ctypes.c_void_p), ("p_start", ctypes.c_void_p), ("p_target", ctypes.c_void_p),
                ("gamma", ctypes.c_void_p), ("endpoints", ctypes.c_void_p), ("status", ctypes.c_void_p),
                ("info", ctypes.c_void_p), ("start_set", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "batches", "tracks_completed",
                                              "latencies", "peak_bytes")] + \
               [(k, ctypes.c_double) for k in ("wall_s", "mean_ms", "p50_ms", "p99_ms", "max_ms")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_server_bound = False


def _bind_server():
    global _server_bound
    if _server_bound:
        return
    L = lib()
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    L.hc_server_default_opts.restype = None
    L.hc_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
    L.hc_server_create.restype = ctypes.c_int
    L.hc_server_create.argtypes = [P, ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]
    L.hc_server_submit.restype = ctypes.c_int
    L.hc_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(I64)]
    L.hc_server_add_start_set.restype = ctypes.c_int
    L.hc_server_add_start_set.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.POINTER(P)]
    L.hc_server_poll.restype = ctypes.c_int
    L.hc_server_poll.argtypes = [P, I64, ctypes.POINTER(ctypes.c_int32)]
    L.hc_server_wait.restype = ctypes.c_int
    L.hc_server_wait.argtypes = [P, I64]
    L.hc_server_get_stats.restype = ctypes.c_int
    L.hc_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.hc_server_reset_stats.restype = ctypes.c_int
    L.hc_server_reset_stats.argtypes = [P]
    L.hc_server_destroy.restype = ctypes.c_int
    L.hc_server_destroy.argtypes = [P]
    _server_bound = True


class StartSet:
    """A start set resident on a server's device (hc_server_add_start_set)."""

    def __init__(self, handle, n_start: int):
        self.handle = handle
        self.n_start = n_start


class Server:
    """hc_server_*: continuous batching of host-buffer solve requests."""

    def __init__(self, ctx: Context, max_inflight: int = 3, max_batch_requests: int = 64,
                 hbm_budget: int = 8 << 30, opts: Optional[Opts] = None):
        _bind_server()
        so = ServerOpts()
        lib().hc_server_default_opts(ctypes.byref(so))
        so.max_inflight = max_inflight
        so.max_batch_requests = max_batch_requests
        so.hbm_budget = hbm_budget
        if opts is not None:
            so.opts = opts
        h = ctypes.c_void_p()
        _check(lib().hc_server_create(ctx.handle, ctypes.byref(so), ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self._out = {}

    def add_start_set(self, s: System, start, p_start=None) -> "StartSet":
        """hc_server_add_start_set: start points [n_start, n] (and p_start) kept on
        the device for requests that name the returned set."""
        st_pts = np.ascontiguousarray(start, np.complex128).reshape(-1, s.n)
        ps = None if p_start is None else np.ascontiguousarray(p_start, np.complex128)
        h = ctypes.c_void_p()
        _check(lib().hc_server_add_start_set(self.handle, s.handle, _ptr(st_pts), st_pts.shape[0], _ptr(ps),
                                             ctypes.byref(h)))
        return StartSet(h, st_pts.shape[0])

    def submit(self, s: System, p_target, gamma=None, start=None, p_start=None, n_start=None,
               with_info: bool = False, start_set: "Optional[StartSet]" = None) -> int:
        p = np.ascontiguousarray(p_target, np.complex128)
        if p.ndim == 1:
            p = p[None, :]
        n_inst = p.shape[0]
        g = None if gamma is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(gamma, np.complex128), (n_inst,)))
        st_pts = None if start is None else np.ascontiguousarray(start, np.complex128).reshape(-1, s.n)
        if n_start is None:
            n_start = start_set.n_start if start_set is not None else \
                s.bezout if st_pts is None else st_pts.shape[0]
        ps = None if p_start is None else np.ascontiguousarray(p_start, np.complex128)
        ep = np.zeros((n_inst, n_start, s.n), np.complex128)
        status = np.zeros((n_inst, n_start), np.int32)
        info = np.zeros((n_inst, n_start), INFO_DTYPE) if with_info else None
        r = Request(s.handle, n_start, n_inst, _ptr(st_pts), _ptr(ps), _ptr(p), _ptr(g), _ptr(ep), _ptr(status),
                    _ptr(info), None if start_set is None else start_set.handle)
        t = ctypes.c_int64()
        _check(lib().hc_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._out[t.value] = (ep, status, info)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(lib().hc_server_poll(self.handle, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int):
        _check(lib().hc_server_wait(self.handle, ticket))
        return self._out.pop(ticket)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().hc_server_get_stats(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        _check(lib().hc_server_reset_stats(self.handle))

    def close(self):
        if self.handle:
            _check(lib().hc_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
