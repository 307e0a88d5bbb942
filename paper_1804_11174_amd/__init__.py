"""Python binding of libkdepic.so: the MI355X von Mises KDE hot path.

The functions named ``kde_*`` mirror the C entry points of ``include/kde.h``
one to one: they only marshal arguments (torch tensors on the GPU supply
device pointers, torch's current stream supplies the HIP stream) and raise
``KdeError`` when a call returns a non-zero status. Every step of the path
runs in the library's HIP kernels; there is no fallback of any kind. If the
shared library has not been built, ``require_library()`` (called by every
entry point) raises.

Convenience wrappers (``cv_scan``, ``deposit``, ``gather``,
``adapt_widths``) allocate outputs and workspace with torch and call the
``kde_*`` functions.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libkdepic.so")

KDE_F64, KDE_F32 = 0, 1
KDE_SHAPE_VONMISES, KDE_SHAPE_TRIANGLE = 0, 1
KDE_OP_CV_SCAN, KDE_OP_DEPOSIT, KDE_OP_GATHER, KDE_OP_ADAPT = 0, 1, 2, 3
KDE_OP_CV_FOURIER, KDE_OP_CV_REFINE, KDE_OP_ADAPT_EXACT = 4, 5, 6
KDE_MAX_FOURIER_KAPPA = 1e6
KDE_MAX_KAPPAS = 64

_lib = None


class KdeError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status} ({message})")
        self.status = status


class kde_domain(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("M", ctypes.c_int32), ("prec", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class kde_batch_set(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("x", ctypes.c_void_p), ("L", ctypes.c_double), ("M", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_cv", ctypes.c_int64), ("cv", ctypes.c_void_p), ("pilot", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("kappa_i", ctypes.c_void_p), ("kappa_star", ctypes.c_void_p)]


class kde_pic_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("L", ctypes.c_double), ("M", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("dt", ctypes.c_double), ("B", ctypes.c_int32), ("n_cv", ctypes.c_int32),
                ("kappas_h", ctypes.POINTER(ctypes.c_double)), ("alpha", ctypes.c_double),
                ("p_threshold", ctypes.c_double), ("adjust_rate", ctypes.c_double), ("method", ctypes.c_int32),
                ("history", ctypes.c_int32)]


class kde_session_info(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("p_th", ctypes.c_double), ("h_opt", ctypes.c_double),
                ("h_target", ctypes.c_double), ("kappa_star", ctypes.c_double), ("last_a2", ctypes.c_double),
                ("last_p", ctypes.c_double), ("fired", ctypes.c_int64), ("numeric", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class kde_server_config(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("B", ctypes.c_int32), ("kappas_h", ctypes.POINTER(ctypes.c_double)),
                ("alpha", ctypes.c_double), ("n_cv", ctypes.c_int64), ("nslots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("large_slots", ctypes.c_int32), ("large_terms", ctypes.c_double)]


class kde_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("latency_s", ctypes.c_double),
                ("queue_s", ctypes.c_double), ("run_s", ctypes.c_double), ("steps", ctypes.c_int64)]


class kde_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("mean_batch", ctypes.c_double), ("p50_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("requests_per_s", ctypes.c_double), ("pair_evals", ctypes.c_double),
                ("particles", ctypes.c_double), ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("session_steps", ctypes.c_int64), ("session_p50_s", ctypes.c_double),
                ("session_p99_s", ctypes.c_double)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_dom_p = ctypes.POINTER(kde_domain)

_SIGNATURES = {
    "kde_abi_version": (_i32, []),
    "kde_status_str": (ctypes.c_char_p, [_i32]),
    "kde_last_error": (ctypes.c_char_p, []),
    "kde_numeric_check": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32)]),
    "kde_workspace_size": (_i32, [_i32, _dom_p, _i64, _i32, ctypes.POINTER(_sz)]),
    "kde_cv_scan": (_i32, [_dom_p, _i64, _vp, _i32, ctypes.POINTER(_dbl), _vp, _vp, _vp, _vp, _sz, _vp]),
    "kde_cv_scan_noalloc": (_i32, [_dom_p, _i64, _vp, _i32, ctypes.POINTER(_dbl), _vp, _vp, _vp, _vp]),
    "kde_deposit": (_i32, [_dom_p, _i64, _vp, _vp, _dbl, _vp, _vp, _sz, _vp]),
    "kde_gather": (_i32, [_dom_p, _i64, _vp, _vp, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "kde_adapt_widths": (_i32, [_dom_p, _i64, _vp, _vp, _dbl, _dbl, _vp, _vp, _vp, _vp, _sz, _vp]),
    "kde_cv_scan_fourier": (_i32, [_dom_p, _i64, _vp, _i32, ctypes.POINTER(_dbl), _vp, _vp, _vp, _vp, _sz, _vp]),
    "kde_cv_refine": (_i32, [_dom_p, _i64, _vp, _i32, ctypes.POINTER(_dbl), _vp, _vp, _vp, _vp, _sz, _vp]),
    "kde_adapt_widths_exact": (_i32, [_dom_p, _i64, _vp, _dbl, _dbl, _vp, _vp, _vp, _vp, _sz, _vp]),
    "kde_timing_enable": (_i32, [_i32]),
    "kde_timing_reset": (_i32, []),
    "kde_timing_read": (_i32, [_i32, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "kde_probe_peak": (_i32, [_i32, _i32, _i64, _vp, _vp]),
    "kde_tune_set": (_i32, [_i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "kde_tune_get": (_i32, [_i32, _i64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "kde_batch_plan": (_i32, [ctypes.POINTER(kde_batch_set), _i32, _i32, _i32, ctypes.POINTER(_dbl), _dbl,
                              ctypes.POINTER(_vp)]),
    "kde_batch_workspace_size": (_i32, [_vp, ctypes.POINTER(_sz)]),
    "kde_batch_run": (_i32, [_vp, _vp, _sz, _vp]),
    "kde_batch_status": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), _vp]),
    "kde_batch_destroy": (_i32, [_vp]),
    "kde_session_bytes": (_i32, [ctypes.POINTER(kde_pic_params), ctypes.POINTER(_sz)]),
    "kde_session_create": (_i32, [ctypes.POINTER(kde_pic_params), _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "kde_session_step": (_i32, [_vp, _i32]),
    "kde_session_state": (_i32, [_vp, ctypes.POINTER(kde_session_info)]),
    "kde_session_read": (_i32, [_vp, _i32, _vp]),
    "kde_session_save": (_i32, [_vp, _vp, ctypes.POINTER(_sz)]),
    "kde_session_restore": (_i32, [_vp, _vp, _sz]),
    "kde_session_destroy": (_i32, [_vp]),
    "kde_ad_pvalue": (_i32, [_dbl, ctypes.POINTER(_dbl)]),
    "kde_damping_rate": (_i32, [ctypes.POINTER(_dbl), _i64, _dbl, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]),
    "kde_server_create": (_i32, [ctypes.POINTER(kde_server_config), _vp, _sz, ctypes.POINTER(_vp)]),
    "kde_server_request_bytes": (_i32, [_vp, ctypes.POINTER(kde_batch_set), ctypes.POINTER(_sz)]),
    "kde_server_submit": (_i32, [_vp, ctypes.POINTER(kde_batch_set), _vp, ctypes.POINTER(ctypes.c_uint64)]),
    "kde_server_attach": (_i32, [_vp, _vp, _i64, ctypes.POINTER(ctypes.c_uint64)]),
    "kde_server_cancel": (_i32, [_vp, ctypes.c_uint64]),
    "kde_server_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(kde_result)]),
    "kde_server_wait": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(kde_result)]),
    "kde_server_drain": (_i32, [_vp]),
    "kde_server_stats": (_i32, [_vp, ctypes.POINTER(kde_server_stats_t)]),
    "kde_server_destroy": (_i32, [_vp]),
}

KDE_SESSION_X, KDE_SESSION_V, KDE_SESSION_KAPPA, KDE_SESSION_RHO, KDE_SESSION_E = 0, 1, 2, 3, 4
KDE_SESSION_ENERGY = 5
KDE_PIC_KDE, KDE_PIC_STANDARD = 0, 1
KDE_E_INVALID_ARG, KDE_E_WORKSPACE, KDE_E_BUDGET, KDE_E_AGAIN, KDE_E_NOT_FOUND = 1, 2, 3, 4, 5
KDE_E_HIP, KDE_E_NUMERIC, KDE_E_INTERNAL, KDE_E_CANCELLED = 6, 7, 8, 9
KDE_NUMERIC_POSITION, KDE_NUMERIC_CONCENTRATION = 1, 2

TUNE_FILE = os.path.join(HERE, "tune_gfx950.json")

KDE_KERNEL_CV_PAIRS, KDE_KERNEL_DEPOSIT, KDE_KERNEL_GATHER, KDE_KERNEL_ADAPT = 0, 1, 2, 3
KDE_KERNEL_MOMENTS, KDE_KERNEL_PROBE = 4, 5
KDE_PROBE_FMA_F64, KDE_PROBE_FMA_F32, KDE_PROBE_EXP_F32, KDE_PROBE_ADD_F64 = 0, 1, 2, 3

EXPORTED = tuple(_SIGNATURES)


def library_path() -> str:
    return LIB_PATH


def require_library():
    """Load libkdepic.so (once) and return it; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libkdepic.so is not built ({LIB_PATH}); run "
                           "`python -m paper_1804_11174_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    if os.path.exists(TUNE_FILE):
        load_tuning(TUNE_FILE)
    return lib


def load_tuning(path: str):
    """Install an autotuned pair-kernel table (JSON written by autotune.py)."""
    import json
    with open(path) as f:
        table = json.load(f)
    for name, prec in (("f64", KDE_F64), ("f32", KDE_F32)):
        rows = table.get(name)
        if rows:
            kde_tune_set(prec, [r["n_max"] for r in rows], [r["chunk"] for r in rows],
                         [r.get("group", 0) for r in rows])


def _check(status: int, where: str):
    if status != 0:
        lib = require_library()
        msg = lib.kde_last_error().decode() or lib.kde_status_str(status).decode()
        raise KdeError(status, where, msg)


# ------------------------------------------------------------ marshalling

def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _domain(L: float, M: int, prec: int, shape: int = KDE_SHAPE_VONMISES) -> kde_domain:
    return kde_domain(float(L), int(M), int(prec), int(shape), 0)


def prec_of(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return KDE_F64
    if t.dtype == torch.float32:
        return KDE_F32
    raise ValueError(f"particle arrays must be float64 or float32 (got {t.dtype})")


# ------------------------------------------------------- C entry points

def kde_abi_version() -> int:
    return int(require_library().kde_abi_version())


def kde_status_str(status: int) -> str:
    return require_library().kde_status_str(int(status)).decode()


def kde_last_error() -> str:
    return require_library().kde_last_error().decode()


def kde_numeric_check(stream=None) -> int:
    """Wait for the stream and take the plain calls' numeric status word
    (KDE_NUMERIC_* bits; 0 when no non-finite value was seen since the last
    check on this device). Returns the bits; does not raise."""
    flags = ctypes.c_uint32(0)
    st = require_library().kde_numeric_check(_stream(stream), ctypes.byref(flags))
    if st not in (0, KDE_E_NUMERIC):
        _check(st, "kde_numeric_check")
    return int(flags.value)


def kde_workspace_size(op: int, dom: kde_domain, N: int, B: int = 0) -> int:
    lib = require_library()
    out = _sz(0)
    _check(lib.kde_workspace_size(int(op), ctypes.byref(dom), int(N), int(B), ctypes.byref(out)),
           "kde_workspace_size")
    return int(out.value)


def kde_cv_scan(dom, N, x, kappas_h, cv, sums, argmin, ws, ws_bytes, stream=None):
    lib = require_library()
    k = np.ascontiguousarray(np.asarray(kappas_h, dtype=np.float64))
    kp = k.ctypes.data_as(ctypes.POINTER(_dbl))
    _check(lib.kde_cv_scan(ctypes.byref(dom), int(N), _ptr(x), int(k.shape[0]), kp, _ptr(cv), _ptr(sums),
                           _ptr(argmin), ws, int(ws_bytes), _stream(stream)), "kde_cv_scan")


def kde_cv_scan_noalloc(dom, N, x, kappas_h, cv, sums, argmin, stream=None):
    lib = require_library()
    k = np.ascontiguousarray(np.asarray(kappas_h, dtype=np.float64))
    kp = k.ctypes.data_as(ctypes.POINTER(_dbl))
    _check(lib.kde_cv_scan_noalloc(ctypes.byref(dom), int(N), _ptr(x), int(k.shape[0]), kp, _ptr(cv), _ptr(sums),
                                   _ptr(argmin), _stream(stream)), "kde_cv_scan_noalloc")


def kde_cv_scan_fourier(dom, N, x, kappas_h, cv, sums, argmin, ws, ws_bytes, stream=None):
    lib = require_library()
    k = np.ascontiguousarray(np.asarray(kappas_h, dtype=np.float64))
    kp = k.ctypes.data_as(ctypes.POINTER(_dbl))
    _check(lib.kde_cv_scan_fourier(ctypes.byref(dom), int(N), _ptr(x), int(k.shape[0]), kp, _ptr(cv), _ptr(sums),
                                   _ptr(argmin), ws, int(ws_bytes), _stream(stream)), "kde_cv_scan_fourier")


def kde_cv_refine(dom, N, x, kappas_h, result, cv, argmin, ws, ws_bytes, stream=None):
    lib = require_library()
    k = np.ascontiguousarray(np.asarray(kappas_h, dtype=np.float64))
    kp = k.ctypes.data_as(ctypes.POINTER(_dbl))
    _check(lib.kde_cv_refine(ctypes.byref(dom), int(N), _ptr(x), int(k.shape[0]), kp, _ptr(result), _ptr(cv),
                             _ptr(argmin), ws, int(ws_bytes), _stream(stream)), "kde_cv_refine")


def kde_adapt_widths_exact(dom, N, x, kappa_star, alpha, kappa_out, log_geomean, n_floored, ws, ws_bytes,
                           stream=None):
    lib = require_library()
    _check(lib.kde_adapt_widths_exact(ctypes.byref(dom), int(N), _ptr(x), float(kappa_star), float(alpha),
                                      _ptr(kappa_out), _ptr(log_geomean), _ptr(n_floored), ws, int(ws_bytes),
                                      _stream(stream)), "kde_adapt_widths_exact")


def kde_deposit(dom, N, x, kappa_i, kappa, rho, ws, ws_bytes, stream=None):
    lib = require_library()
    _check(lib.kde_deposit(ctypes.byref(dom), int(N), _ptr(x), _ptr(kappa_i), float(kappa), _ptr(rho), ws,
                           int(ws_bytes), _stream(stream)), "kde_deposit")


def kde_gather(dom, N, x, kappa_i, kappa, field, out, ws, ws_bytes, stream=None):
    lib = require_library()
    _check(lib.kde_gather(ctypes.byref(dom), int(N), _ptr(x), _ptr(kappa_i), float(kappa), _ptr(field), _ptr(out),
                          ws, int(ws_bytes), _stream(stream)), "kde_gather")


def kde_adapt_widths(dom, N, x, pilot, kappa_star, alpha, kappa_out, log_geomean, n_floored, ws, ws_bytes,
                     stream=None):
    lib = require_library()
    _check(lib.kde_adapt_widths(ctypes.byref(dom), int(N), _ptr(x), _ptr(pilot), float(kappa_star), float(alpha),
                                _ptr(kappa_out), _ptr(log_geomean), _ptr(n_floored), ws, int(ws_bytes),
                                _stream(stream)), "kde_adapt_widths")


def kde_tune_set(prec: int, n_max, chunk, group=None):
    """Pair-kernel table: entry k (N <= n_max[k]) evaluates chunk[k]
    concentrations per pass and gives each workgroup group[k] of them
    (0 = all)."""
    lib = require_library()
    n = len(n_max)
    a = (_i64 * n)(*[int(v) for v in n_max])
    b = (_i32 * n)(*[int(v) for v in chunk])
    g = None if group is None else (_i32 * n)(*[int(v) for v in group])
    _check(lib.kde_tune_set(int(prec), n, a, b, g), "kde_tune_set")


def kde_tune_get(prec: int, N: int) -> Tuple[int, int]:
    """``(chunk, group)`` of the table entry used for N."""
    c, g = _i32(0), _i32(0)
    _check(require_library().kde_tune_get(int(prec), int(N), ctypes.byref(c), ctypes.byref(g)), "kde_tune_get")
    return int(c.value), int(g.value)


def kde_batch_plan(sets, prec: int, kappas, alpha: float = 0.5) -> int:
    """Plan a batch from a list of ``kde_batch_set``; returns the handle."""
    lib = require_library()
    arr = (kde_batch_set * len(sets))(*sets)
    k = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64))
    h = _vp()
    _check(lib.kde_batch_plan(arr, len(sets), int(prec), int(k.shape[0]), k.ctypes.data_as(ctypes.POINTER(_dbl)),
                              float(alpha), ctypes.byref(h)), "kde_batch_plan")
    return h.value


def kde_batch_workspace_size(handle: int) -> int:
    out = _sz(0)
    _check(require_library().kde_batch_workspace_size(handle, ctypes.byref(out)), "kde_batch_workspace_size")
    return int(out.value)


def kde_batch_run(handle: int, ws, ws_bytes: int, stream=None):
    _check(require_library().kde_batch_run(handle, ws, int(ws_bytes), _stream(stream)), "kde_batch_run")


def kde_batch_status(handle: int, nsets: int, stream=None):
    """Per-set KDE_NUMERIC_* bits of the last run (waits for the stream)."""
    flags = (ctypes.c_uint32 * nsets)()
    st = require_library().kde_batch_status(handle, flags, _stream(stream))
    if st not in (0, KDE_E_NUMERIC):
        _check(st, "kde_batch_status")
    return [int(f) for f in flags]


def kde_batch_destroy(handle: int):
    _check(require_library().kde_batch_destroy(handle), "kde_batch_destroy")


class Batch:
    """Many particle sets through the whole path in one graph launch.

    ``xs`` are GPU tensors (all float64 or all float32), ``Ls`` and ``Ms``
    their periods and grids. Outputs are allocated here: ``cv[s]`` (B),
    ``pilot[s]`` (M), ``rho[s]`` (M), ``kappa_i[s]`` (N), ``kappa_star``
    (one per set)."""

    def __init__(self, xs, Ls, Ms, kappas, alpha: float = 0.5, n_cv=None):
        import torch
        self.prec = prec_of(xs[0])
        dev = xs[0].device
        self.kappas = np.asarray(kappas, dtype=np.float64)
        B = self.kappas.shape[0]
        self.xs = list(xs)
        self.cv = [torch.empty(B, dtype=torch.float64, device=dev) for _ in xs]
        self.pilot = [torch.empty(int(M), dtype=torch.float64, device=dev) for M in Ms]
        self.rho = [torch.empty(int(M), dtype=torch.float64, device=dev) for M in Ms]
        self.kappa_i = [torch.empty(x.shape[0], dtype=x.dtype, device=dev) for x in xs]
        self.kappa_star = torch.empty(len(xs), dtype=torch.float64, device=dev)
        sets = []
        for s, (x, L, M) in enumerate(zip(xs, Ls, Ms)):
            if prec_of(x) != self.prec:
                raise ValueError("all sets of a batch share one precision")
            ncv = 0 if n_cv is None else min(int(n_cv), int(x.shape[0]))
            sets.append(kde_batch_set(int(x.shape[0]), _ptr(x), float(L), int(M), 0, ncv, _ptr(self.cv[s]),
                                      _ptr(self.pilot[s]), _ptr(self.rho[s]), _ptr(self.kappa_i[s]),
                                      self.kappa_star.data_ptr() + 8 * s))
        self.handle = kde_batch_plan(sets, self.prec, self.kappas, alpha)
        self.ws = Workspace(dev)
        self.ws.get(kde_batch_workspace_size(self.handle))

    def run(self, stream=None):
        kde_batch_run(self.handle, self.ws.ptr, self.ws.bytes, stream)

    def close(self):
        if self.handle:
            kde_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- sessions

def _params(N, L, M, prec, dt, kappas, n_cv, alpha=0.5, p_threshold=0.01, adjust_rate=0.05,
            method=KDE_PIC_KDE, history=0):
    k = np.ascontiguousarray(np.asarray(kappas if kappas is not None else [1.0], dtype=np.float64))
    p = kde_pic_params(int(N), float(L), int(M), int(prec), float(dt), int(k.shape[0]), int(n_cv),
                       k.ctypes.data_as(ctypes.POINTER(_dbl)), float(alpha), float(p_threshold), float(adjust_rate),
                       int(method), int(history))
    return p, k


def kde_damping_rate(energy, dt):
    """The damping rate of a field-energy history (host array) as the
    library computes it: ``(rate, (p1, p2))``."""
    e = np.ascontiguousarray(np.asarray(energy, dtype=np.float64))
    rate = _dbl(0.0)
    peaks = (_i64 * 2)()
    _check(require_library().kde_damping_rate(e.ctypes.data_as(ctypes.POINTER(_dbl)), int(e.shape[0]), float(dt),
                                              ctypes.byref(rate), peaks), "kde_damping_rate")
    return rate.value, (int(peaks[0]), int(peaks[1]))


damping_rate = kde_damping_rate


def kde_session_bytes(params) -> int:
    out = _sz(0)
    _check(require_library().kde_session_bytes(ctypes.byref(params), ctypes.byref(out)), "kde_session_bytes")
    return int(out.value)


def kde_session_create(params, x0, v0, arena, arena_bytes, stream=None) -> int:
    h = _vp()
    _check(require_library().kde_session_create(ctypes.byref(params), _ptr(x0), _ptr(v0), arena, int(arena_bytes),
                                                _stream(stream), ctypes.byref(h)), "kde_session_create")
    return h.value


def kde_session_step(handle, nsteps: int = 1):
    _check(require_library().kde_session_step(handle, int(nsteps)), "kde_session_step")


def kde_session_state(handle) -> dict:
    info = kde_session_info()
    _check(require_library().kde_session_state(handle, ctypes.byref(info)), "kde_session_state")
    return {f: getattr(info, f) for f, _ in kde_session_info._fields_}


def kde_session_read(handle, what: int, dst):
    _check(require_library().kde_session_read(handle, int(what), _ptr(dst)), "kde_session_read")


def kde_session_save(handle) -> bytes:
    lib = require_library()
    n = _sz(0)
    _check(lib.kde_session_save(handle, None, ctypes.byref(n)), "kde_session_save")
    buf = ctypes.create_string_buffer(n.value)
    _check(lib.kde_session_save(handle, buf, ctypes.byref(n)), "kde_session_save")
    return buf.raw[:n.value]


def kde_session_restore(handle, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(require_library().kde_session_restore(handle, buf, len(blob)), "kde_session_restore")


def kde_session_destroy(handle):
    _check(require_library().kde_session_destroy(handle), "kde_session_destroy")


def kde_ad_pvalue(a2: float) -> float:
    out = _dbl(0.0)
    _check(require_library().kde_ad_pvalue(float(a2), ctypes.byref(out)), "kde_ad_pvalue")
    return float(out.value)


class Session:
    """A resident PIC session; x0, v0 are GPU tensors (float64 or float32)."""

    def __init__(self, x0, v0, L, M, dt, kappas=None, n_cv=2, alpha=0.5, p_threshold=0.01, adjust_rate=0.05,
                 method=KDE_PIC_KDE, history=0):
        import torch
        self.N, self.M, self.dtype, self.device = x0.shape[0], int(M), x0.dtype, x0.device
        self.history = int(history)
        self.params, self._k = _params(self.N, L, M, prec_of(x0), dt, kappas, n_cv, alpha, p_threshold, adjust_rate,
                                       method, history)
        nbytes = kde_session_bytes(self.params)
        self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=x0.device)
        base = self._arena.data_ptr()
        self.handle = kde_session_create(self.params, x0, v0, (base + 255) // 256 * 256, nbytes)

    def step(self, n=1):
        kde_session_step(self.handle, n)

    def state(self):
        return kde_session_state(self.handle)

    def read(self, what):
        import torch
        if what in (KDE_SESSION_RHO, KDE_SESSION_E):
            out = torch.empty(self.M, dtype=torch.float64, device=self.device)
        elif what == KDE_SESSION_ENERGY:
            n = min(int(self.state()["step"]), self.history)
            out = torch.empty(n, dtype=torch.float64, device=self.device)
            if n == 0:
                return out
        else:
            out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        kde_session_read(self.handle, what, out)
        return out

    def save(self):
        return kde_session_save(self.handle)

    def restore(self, blob):
        kde_session_restore(self.handle, blob)

    def close(self):
        if self.handle:
            kde_session_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- server

def kde_server_create(cfg, arena, budget) -> int:
    h = _vp()
    _check(require_library().kde_server_create(ctypes.byref(cfg), arena, int(budget), ctypes.byref(h)),
           "kde_server_create")
    return h.value


def kde_server_request_bytes(handle, req) -> int:
    out = _sz(0)
    _check(require_library().kde_server_request_bytes(handle, ctypes.byref(req), ctypes.byref(out)),
           "kde_server_request_bytes")
    return int(out.value)


def kde_server_submit(handle, req, stream=None) -> int:
    t = ctypes.c_uint64(0)
    _check(require_library().kde_server_submit(handle, ctypes.byref(req), _stream(stream), ctypes.byref(t)),
           "kde_server_submit")
    return int(t.value)


def kde_server_attach(handle, session_handle, nsteps: int) -> int:
    t = ctypes.c_uint64(0)
    _check(require_library().kde_server_attach(handle, session_handle, int(nsteps), ctypes.byref(t)),
           "kde_server_attach")
    return int(t.value)


def kde_server_cancel(handle, ticket: int) -> bool:
    """True when the queued request was withdrawn or the attached session
    detaches (after its step in flight), False when the request already runs."""
    st = require_library().kde_server_cancel(handle, ctypes.c_uint64(ticket))
    if st == KDE_E_AGAIN:
        return False
    _check(st, "kde_server_cancel")
    return True


def kde_server_poll(handle, ticket: int):
    """The result as a dict once done (``status`` 0, or the status it ended
    with: numeric, cancelled, HIP), else None while pending."""
    r = kde_result()
    st = require_library().kde_server_poll(handle, ctypes.c_uint64(ticket), ctypes.byref(r))
    if st == KDE_E_AGAIN:
        return None
    if st not in (0, KDE_E_NUMERIC, KDE_E_CANCELLED, KDE_E_HIP):
        _check(st, "kde_server_poll")
    return {f: getattr(r, f) for f, _ in kde_result._fields_}


def kde_server_wait(handle, ticket: int) -> dict:
    """Block until the ticket completes; its result as kde_server_poll's."""
    r = kde_result()
    st = require_library().kde_server_wait(handle, ctypes.c_uint64(ticket), ctypes.byref(r))
    if st not in (0, KDE_E_NUMERIC, KDE_E_CANCELLED, KDE_E_HIP):
        _check(st, "kde_server_wait")
    return {f: getattr(r, f) for f, _ in kde_result._fields_}


def kde_server_drain(handle):
    _check(require_library().kde_server_drain(handle), "kde_server_drain")


def kde_server_stats(handle) -> dict:
    st = kde_server_stats_t()
    _check(require_library().kde_server_stats(handle, ctypes.byref(st)), "kde_server_stats")
    return {f: getattr(st, f) for f, _ in kde_server_stats_t._fields_}


def kde_server_destroy(handle):
    _check(require_library().kde_server_destroy(handle), "kde_server_destroy")


class Server:
    """Continuous-batching server of KDE solves over a torch-owned arena."""

    def __init__(self, kappas, prec=KDE_F32, budget_bytes=256 << 20, nslots=4, max_batch=16, n_cv=65536,
                 alpha=0.5, device="cuda", large_slots=0, large_terms=0.0):
        import torch
        self._k = np.ascontiguousarray(np.asarray(kappas, dtype=np.float64))
        self.cfg = kde_server_config(int(prec), int(self._k.shape[0]), self._k.ctypes.data_as(ctypes.POINTER(_dbl)),
                                     float(alpha), int(n_cv), int(nslots), int(max_batch), int(large_slots),
                                     float(large_terms))
        self._arena = torch.empty(int(budget_bytes) + 256, dtype=torch.uint8, device=device)
        base = self._arena.data_ptr()
        self.handle = kde_server_create(self.cfg, (base + 255) // 256 * 256, int(budget_bytes))
        self.B = int(self._k.shape[0])

    @staticmethod
    def request(x, L, M, outputs, n_cv=0):
        """A kde_batch_set for positions x with output tensors
        (cv[B], pilot[M], rho[M], kappa_i[N], kappa_star[1])."""
        cv, pilot, rho, k_i, ks = outputs
        return kde_batch_set(int(x.shape[0]), _ptr(x), float(L), int(M), 0, int(n_cv), _ptr(cv), _ptr(pilot),
                             _ptr(rho), _ptr(k_i), _ptr(ks))

    def submit(self, req, stream=None) -> int:
        return kde_server_submit(self.handle, req, stream)

    def attach(self, session, nsteps: int) -> int:
        """Hand a Session to the server for nsteps steps; poll the ticket."""
        return kde_server_attach(self.handle, session.handle, nsteps)

    def cancel(self, ticket) -> bool:
        return kde_server_cancel(self.handle, ticket)

    def poll(self, ticket):
        return kde_server_poll(self.handle, ticket)

    def wait(self, ticket):
        return kde_server_wait(self.handle, ticket)

    def drain(self):
        kde_server_drain(self.handle)

    def stats(self):
        return kde_server_stats(self.handle)

    def close(self):
        if self.handle:
            kde_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kde_timing_enable(on: bool):
    _check(require_library().kde_timing_enable(1 if on else 0), "kde_timing_enable")


def kde_timing_reset():
    _check(require_library().kde_timing_reset(), "kde_timing_reset")


def kde_timing_read(kernel_id: int) -> Tuple[float, int]:
    """``(total_ms, launches)`` accumulated for one kernel since the last reset."""
    ms = _dbl(0.0)
    n = _i64(0)
    _check(require_library().kde_timing_read(int(kernel_id), ctypes.byref(ms), ctypes.byref(n)), "kde_timing_read")
    return float(ms.value), int(n.value)


def kde_probe_peak(kind: int, blocks: int, iters: int, out, stream=None) -> None:
    """Launch the issue-rate probe: blocks x 256 threads, each running 8
    dependency chains of ``iters`` steps of one instruction kind; ``out`` is
    a device tensor of blocks x 256 doubles."""
    import torch
    if out.dtype != torch.float64 or out.numel() < blocks * 256 or not out.is_cuda:
        raise ValueError("out must be a device float64 tensor of at least blocks x 256 elements")
    _check(require_library().kde_probe_peak(int(kind), int(blocks), int(iters), _ptr(out), _stream(stream)),
           "kde_probe_peak")


# ------------------------------------------------------- workspace helper

class Workspace:
    """A 256-byte aligned device buffer that grows on demand (torch memory)."""

    def __init__(self, device="cuda"):
        self.device = device
        self._buf = None
        self.ptr = None
        self.bytes = 0

    def get(self, nbytes: int) -> Tuple[Optional[int], int]:
        import torch
        if nbytes == 0:
            return None, 0
        if nbytes > self.bytes:
            self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self._buf.data_ptr()
            self.ptr = (base + 255) // 256 * 256
            self.bytes = nbytes
        return self.ptr, self.bytes


_default_ws = {}


def _ws(nbytes: int, device) -> Tuple[Optional[int], int]:
    import torch
    key = torch.device(device).index if torch.device(device).index is not None else torch.cuda.current_device()
    w = _default_ws.setdefault(key, Workspace(f"cuda:{key}"))
    return w.get(nbytes)


# ------------------------------------------------------ convenience layer

def cv_scan(x, L: float, kappas, ws: Optional[Workspace] = None, stream=None, shape: int = KDE_SHAPE_VONMISES):
    """CV objective over ``kappas`` (ascending; half-widths for the
    triangle shape) for positions ``x`` (GPU tensor, float64 or float32).
    Returns ``(cv[B], sums[2B], argmin[1])`` as GPU tensors (float64,
    float64, int32)."""
    import torch
    k = np.asarray(kappas, dtype=np.float64)
    dom = _domain(L, 2, prec_of(x), shape)
    n = x.shape[0]
    cv = torch.empty(k.shape[0], dtype=torch.float64, device=x.device)
    sums = torch.empty(2 * k.shape[0], dtype=torch.float64, device=x.device)
    am = torch.empty(1, dtype=torch.int32, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_CV_SCAN, dom, n, k.shape[0])
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_cv_scan(dom, n, x, k, cv, sums, am, ptr, cap, stream)
    return cv, sums, am


def cv_scan_fourier(x, L: float, kappas, ws: Optional[Workspace] = None, stream=None):
    """The CV objective of ``cv_scan`` through the sample's Fourier moments
    (von Mises shape). Returns ``(cv[B], sums[2B], argmin[1])``."""
    import torch
    k = np.asarray(kappas, dtype=np.float64)
    dom = _domain(L, 2, prec_of(x))
    n = x.shape[0]
    cv = torch.empty(k.shape[0], dtype=torch.float64, device=x.device)
    sums = torch.empty(2 * k.shape[0], dtype=torch.float64, device=x.device)
    am = torch.empty(1, dtype=torch.int32, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_CV_FOURIER, dom, n, k.shape[0])
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_cv_scan_fourier(dom, n, x, k, cv, sums, am, ptr, cap, stream)
    return cv, sums, am


def cv_refine(x, L: float, kappas, ws: Optional[Workspace] = None, stream=None):
    """Minimiser of the CV objective in concentration inside the bracket of
    the scan's first minimum. Returns ``(result[5], cv[B], argmin[1])`` with
    result = [kappa*, cv(kappa*), dCV/dlog(kappa) there, steps, b*]."""
    import torch
    k = np.asarray(kappas, dtype=np.float64)
    dom = _domain(L, 2, prec_of(x))
    n = x.shape[0]
    res = torch.empty(5, dtype=torch.float64, device=x.device)
    cv = torch.empty(k.shape[0], dtype=torch.float64, device=x.device)
    am = torch.empty(1, dtype=torch.int32, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_CV_REFINE, dom, n, k.shape[0])
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_cv_refine(dom, n, x, k, res, cv, am, ptr, cap, stream)
    return res, cv, am


def adapt_widths_exact(x, L: float, kappa_star: float, alpha: float = 0.5, ws: Optional[Workspace] = None,
                       stream=None):
    """Per-particle concentrations from the exact pilot at the particles.
    Returns ``(kappa_i, log_geomean[1], n_floored[1])``."""
    import torch
    dom = _domain(L, 2, prec_of(x))
    n = x.shape[0]
    kout = torch.empty(n, dtype=x.dtype, device=x.device)
    lg = torch.empty(1, dtype=torch.float64, device=x.device)
    nf = torch.empty(1, dtype=torch.int64, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_ADAPT_EXACT, dom, n)
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_adapt_widths_exact(dom, n, x, kappa_star, alpha, kout, lg, nf, ptr, cap, stream)
    return kout, lg, nf


def deposit(x, L: float, M: int, kappa: float = 0.0, kappa_i=None, ws: Optional[Workspace] = None,
            stream=None, shape: int = KDE_SHAPE_VONMISES):
    """Grid density (M float64 values) with a global ``kappa`` or per-particle
    ``kappa_i`` (same dtype as ``x``); half-widths for the triangle shape."""
    import torch
    dom = _domain(L, M, prec_of(x), shape)
    n = x.shape[0]
    rho = torch.empty(M, dtype=torch.float64, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_DEPOSIT, dom, n)
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_deposit(dom, n, x, kappa_i, kappa, rho, ptr, cap, stream)
    return rho


def gather(x, L: float, field, kappa: float = 0.0, kappa_i=None, stream=None, shape: int = KDE_SHAPE_VONMISES):
    """Field (M float64 values) interpolated to the particles (dtype of x)."""
    import torch
    M = field.shape[0]
    dom = _domain(L, M, prec_of(x), shape)
    n = x.shape[0]
    out = torch.empty(n, dtype=x.dtype, device=x.device)
    kde_gather(dom, n, x, kappa_i, kappa, field, out, None, 0, stream)
    return out


def adapt_widths(x, L: float, pilot, kappa_star: float, alpha: float = 0.5, ws: Optional[Workspace] = None,
                 stream=None, shape: int = KDE_SHAPE_VONMISES):
    """Per-particle concentrations from a pilot grid. Returns
    ``(kappa_i, log_geomean[1], n_floored[1])``. Defined for the von Mises
    shape only (another ``shape`` raises KdeError)."""
    import torch
    M = pilot.shape[0]
    dom = _domain(L, M, prec_of(x), shape)
    n = x.shape[0]
    kout = torch.empty(n, dtype=x.dtype, device=x.device)
    lg = torch.empty(1, dtype=torch.float64, device=x.device)
    nf = torch.empty(1, dtype=torch.int64, device=x.device)
    nbytes = kde_workspace_size(KDE_OP_ADAPT, dom, n)
    ptr, cap = ws.get(nbytes) if ws is not None else _ws(nbytes, x.device)
    kde_adapt_widths(dom, n, x, pilot, kappa_star, alpha, kout, lg, nf, ptr, cap, stream)
    return kout, lg, nf
