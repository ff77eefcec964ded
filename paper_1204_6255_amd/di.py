"""ctypes binding of libdi (include/di.h), with the same names as the C ABI.

Argument marshalling only: every step of a solve runs in libdi's HIP
kernels. PyTorch tensors may be passed to the *_dev calls (their data_ptr()
and the current HIP stream are forwarded). Loading fails loudly when
libdi.so has not been built; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DI_LIB names another build of the library (the host-sanitizer test's)
LIB_PATH = os.environ.get("DI_LIB") or os.path.join(_HERE, "libdi.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "di.h")

DI_OK, DI_PENDING = 0, 1
DI_E_INVAL, DI_E_UNSORTED, DI_E_DUP, DI_E_RANGE = -1, -2, -3, -4
DI_E_NOMEM, DI_E_NOCONV, DI_E_DEVICE, DI_E_BUSY, DI_E_NOTFOUND = -5, -6, -7, -8, -9
DI_SOP, DI_CYC, DI_PI, DI_GS_ASYNC = 0, 1, 2, 3
DI_FP64, DI_FP32_REFINE, DI_FP32 = 0, 1, 2
DI_STOP_RESID, DI_STOP_PAPER = 0, 1
DI_FLAG_KERNEL_TIMING = 1
DI_FLAG_SERVE_NO_SOLO = 2
DI_FLAG_NO_TUNE = 4
DI_KERNEL_AUTO, DI_KERNEL_PULL, DI_KERNEL_PUSH, DI_KERNEL_WINDOW = 0, 1, 2, 3

STATUS_NAMES = {
    0: "DI_OK", 1: "DI_PENDING", -1: "DI_E_INVAL", -2: "DI_E_UNSORTED", -3: "DI_E_DUP",
    -4: "DI_E_RANGE", -5: "DI_E_NOMEM", -6: "DI_E_NOCONV", -7: "DI_E_DEVICE", -8: "DI_E_BUSY",
    -9: "DI_E_NOTFOUND",
}


class di_opts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("stop", ctypes.c_int32),
        ("max_cycles", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("kernel", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("stream", ctypes.c_void_p),
    ]


class di_stats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int32),
        ("fallback_cycles", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("move_launches", ctypes.c_int32),
        ("edges_pushed", ctypes.c_int64),
        ("nb_iter", ctypes.c_double),
        ("resid_l1", ctypes.c_double),
        ("err_bound", ctypes.c_double),
        ("paper_err", ctypes.c_double),
        ("e", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("move_seconds", ctypes.c_double),
        ("bytes_moved", ctypes.c_double),
        ("move_bytes", ctypes.c_double),
        ("seconds_to_1e9", ctypes.c_double),
        ("queue_seconds", ctypes.c_double),
        ("run_seconds", ctypes.c_double),
        ("readout_seconds", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class di_cycle_rec(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_double),
        ("links", ctypes.c_int64),
        ("selected", ctypes.c_int32),
        ("senders", ctypes.c_int32),
    ]


class di_serve_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("admission_stalls", ctypes.c_int64),
        ("active", ctypes.c_int64),
        ("pending", ctypes.c_int64),
        ("bytes_in_use", ctypes.c_int64),
        ("busy_seconds", ctypes.c_double),
        ("solo_requests", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class DIError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libdi (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing. Build it with `python -c \"import __graft_entry__ as g; g.build()\"` "
            "(hipcc, gfx950); there is no CPU fallback.")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.di_opts_default.argtypes = [P(di_opts)]
    L.di_opts_default.restype = None
    L.di_graph_create.argtypes = [i64, i64, vp, vp, u32, P(vp)]
    L.di_graph_create.restype = i32
    L.di_graph_destroy.argtypes = [vp]
    L.di_graph_destroy.restype = None
    L.di_graph_info.argtypes = [vp, P(i64), P(i64), P(i64), P(i64)]
    L.di_graph_info.restype = i32
    L.di_solve.argtypes = [vp, vp, dbl, dbl, P(di_opts), vp, P(di_stats)]
    L.di_solve.restype = i32
    L.di_solve_dev.argtypes = [vp, vp, dbl, dbl, P(di_opts), vp, P(di_stats)]
    L.di_solve_dev.restype = i32
    L.di_solve_trace_dev.argtypes = [vp, vp, dbl, dbl, P(di_opts), vp, P(di_stats),
                                     P(di_cycle_rec), i32, P(i32)]
    L.di_solve_trace_dev.restype = i32
    L.di_cycles_dev.argtypes = [vp, dbl, i32, vp, vp, i32, P(dbl), vp, P(di_stats)]
    L.di_cycles_dev.restype = i32
    L.di_residual_dev.argtypes = [vp, vp, dbl, vp, vp, P(dbl), vp]
    L.di_residual_dev.restype = i32
    L.di_graph_tuning.argtypes = [vp, P(i32), P(i32), P(i32), P(i32), P(i32), P(i32), P(dbl),
                                  P(dbl), P(dbl)]
    L.di_graph_tuning.restype = i32
    L.di_graph_set_window.argtypes = [vp, i32, i32, i32, i32]
    L.di_graph_set_window.restype = i32
    L.di_residual_dev_noalloc.argtypes = [vp, vp, dbl, vp, vp, P(dbl), vp]
    L.di_residual_dev_noalloc.restype = i32
    L.di_serve_create.argtypes = [ctypes.c_size_t, i32, P(di_opts), P(vp)]
    L.di_serve_create.restype = i32
    L.di_serve_add_graph.argtypes = [vp, vp, i32]
    L.di_serve_add_graph.restype = i32
    L.di_serve_submit.argtypes = [vp, i32, i32, vp, dbl, dbl, P(ctypes.c_uint64)]
    L.di_serve_submit.restype = i32
    L.di_serve_poll.argtypes = [vp, ctypes.c_uint64, vp, P(di_stats)]
    L.di_serve_poll.restype = i32
    L.di_serve_info.argtypes = [vp, P(di_serve_stats)]
    L.di_serve_info.restype = i32
    L.di_serve_destroy.argtypes = [vp]
    L.di_serve_destroy.restype = None
    L.di_solve_batch.argtypes = [vp, i32, vp, dbl, vp, P(di_opts), vp, P(di_stats)]
    L.di_solve_batch.restype = i32
    L.di_solve_batch_dev.argtypes = [vp, i32, vp, dbl, vp, P(di_opts), vp, P(di_stats)]
    L.di_solve_batch_dev.restype = i32
    L.di_last_error.argtypes = []
    L.di_last_error.restype = ctypes.c_char_p
    L.di_version.argtypes = []
    L.di_version.restype = i32
    _lib = L
    return L


def declared_functions() -> list[str]:
    """Names of the functions include/di.h declares."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(di_[a-z0-9_]+)\s*\(", text)))


def di_last_error() -> str:
    return lib().di_last_error().decode(errors="replace")


def di_version() -> int:
    return lib().di_version()


def di_opts_default() -> di_opts:
    o = di_opts()
    lib().di_opts_default(ctypes.byref(o))
    return o


def _check(status: int, allow=(DI_OK,)) -> int:
    if status not in allow:
        raise DIError(status, di_last_error())
    return status


def _ptr(x):
    """Data pointer of a numpy array or torch tensor (None -> NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(x.ctypes.data)


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def di_graph_create(n: int, src, dst, flags: int = 0):
    """Returns (status, handle). src/dst: int32 host arrays."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    h = ctypes.c_void_p()
    st = lib().di_graph_create(int(n), int(src.size), src.ctypes.data, dst.ctypes.data,
                               int(flags), ctypes.byref(h))
    return st, h


def di_graph_destroy(h) -> None:
    if h:
        lib().di_graph_destroy(h)


def di_graph_info(h):
    n, m, nd, nl = (ctypes.c_int64() for _ in range(4))
    _check(lib().di_graph_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(nd), ctypes.byref(nl)))
    return n.value, m.value, nd.value, nl.value


def di_solve(h, B, d: float, tol: float, opts: di_opts | None, X) -> tuple[int, di_stats]:
    """Host arrays: B (n float64, or None for (1-d)/n), X (n float64, written)."""
    st = di_stats()
    status = lib().di_solve(h, _ptr(B), float(d), float(tol),
                            ctypes.byref(opts) if opts is not None else None, _ptr(X), ctypes.byref(st))
    return status, st


def di_solve_dev(h, B_dev, d: float, tol: float, opts: di_opts | None, X_dev) -> tuple[int, di_stats]:
    """Device tensors: B_dev (n float64 or None), X_dev (n float64). The
    current torch stream is used unless opts.stream is set."""
    if opts is None:
        opts = di_opts_default()
    if not opts.stream:
        opts.stream = _current_stream()
    st = di_stats()
    status = lib().di_solve_dev(h, _ptr(B_dev), float(d), float(tol), ctypes.byref(opts), _ptr(X_dev),
                                ctypes.byref(st))
    return status, st


def di_solve_trace_dev(h, B_dev, d: float, tol: float, opts: di_opts | None, X_dev,
                       capacity: int) -> tuple[int, di_stats, list[di_cycle_rec]]:
    """di_solve_dev that also returns the first `capacity` per-cycle records."""
    if opts is None:
        opts = di_opts_default()
    if not opts.stream:
        opts.stream = _current_stream()
    st = di_stats()
    recs = (di_cycle_rec * max(int(capacity), 1))()
    count = ctypes.c_int32(0)
    status = lib().di_solve_trace_dev(h, _ptr(B_dev), float(d), float(tol), ctypes.byref(opts),
                                      _ptr(X_dev), ctypes.byref(st), recs, int(capacity),
                                      ctypes.byref(count))
    return status, st, list(recs[:count.value])


def di_cycles_dev(h, d: float, method: int, F_dev, H_dev, cycles: int, e: float = 0.0, stream=None):
    """Runs `cycles` FP64 cycles in place on device tensors F, H.
    Returns (status, e, stats)."""
    st = di_stats()
    e_c = ctypes.c_double(e)
    status = lib().di_cycles_dev(h, float(d), int(method), _ptr(F_dev), _ptr(H_dev), int(cycles),
                                 ctypes.byref(e_c), stream if stream is not None else _current_stream(),
                                 ctypes.byref(st))
    return status, e_c.value, st


def di_graph_tuning(h):
    """What DI_KERNEL_AUTO runs for DI-SOP on the graph and its window
    configuration: dict(kernel, tile, hubs, grid, rounds, tuned, and the
    tuner's us_default, us_tuned, us_pull per tenfold cut of the
    residual)."""
    v = [ctypes.c_int32() for _ in range(6)]
    u = [ctypes.c_double() for _ in range(3)]
    _check(lib().di_graph_tuning(h, *[ctypes.byref(x) for x in v], *[ctypes.byref(x) for x in u]))
    return {"kernel": {DI_KERNEL_WINDOW: "window", DI_KERNEL_PULL: "pull"}[v[0].value],
            "tile": v[1].value, "hubs": v[2].value, "grid": v[3].value, "rounds": v[4].value,
            "tuned": bool(v[5].value), "us_default": u[0].value, "us_tuned": u[1].value,
            "us_pull": u[2].value}


def di_graph_set_window(h, tile: int, hubs: int, grid_cap: int, rounds: int = 2) -> int:
    """Pins the graph's window-push configuration (no tuning). Returns the
    status."""
    return lib().di_graph_set_window(h, int(tile), int(hubs), int(grid_cap), int(rounds))


def di_residual_dev(h, B_dev, d: float, X_dev, R_dev=None, stream=None):
    """FP64 residual R = B + P.X - X on the device (R_dev may be None).
    Returns (status, |R|_1)."""
    l1 = ctypes.c_double(0.0)
    status = lib().di_residual_dev(h, _ptr(B_dev), float(d), _ptr(X_dev), _ptr(R_dev),
                                   ctypes.byref(l1),
                                   stream if stream is not None else _current_stream())
    return status, l1.value


def di_residual_dev_noalloc(h, B_dev, d: float, X_dev, R_dev=None, stream=None):
    """di_residual_dev without device allocation (its scratch is the
    library's fixed per-device array). Returns (status, |R|_1)."""
    l1 = ctypes.c_double(0.0)
    status = lib().di_residual_dev_noalloc(h, _ptr(B_dev), float(d), _ptr(X_dev), _ptr(R_dev),
                                           ctypes.byref(l1),
                                           stream if stream is not None else _current_stream())
    return status, l1.value


def di_solve_batch(h, k: int, B, d: float, tol, opts=None, X=None):
    """k right-hand sides at once (host arrays). B: (k, n) float64 or None;
    tol: k values. Returns (status, X (k, n), [di_stats] * k)."""
    tol = _tol_array(tol, k)
    n = _graph_n(h) if h else 0
    if B is not None and k > 0:
        B = np.ascontiguousarray(B, dtype=np.float64).reshape(k, n)
    if X is None:
        X = np.empty((max(k, 1), n), np.float64)
    stats = (di_stats * max(k, 1))()
    status = lib().di_solve_batch(h, int(k), _ptr(B), float(d), tol.ctypes.data,
                                  ctypes.byref(opts) if opts is not None else None,
                                  X.ctypes.data, stats)
    return status, X, list(stats)


def di_solve_batch_dev(h, k: int, B_dev, d: float, tol, opts=None, X_dev=None):
    """Device variant (torch tensors of shape (k, n), float64; B_dev may be
    None). opts.stream defaults to the current stream. Returns (status,
    [di_stats] * k)."""
    tol = _tol_array(tol, k)
    if opts is None:
        opts = di_opts_default()
    if not opts.stream:
        opts.stream = _current_stream().value
    stats = (di_stats * max(k, 1))()
    status = lib().di_solve_batch_dev(h, int(k), _ptr(B_dev), float(d), tol.ctypes.data,
                                      ctypes.byref(opts), _ptr(X_dev), stats)
    return status, list(stats)


def di_serve_create(hbm_budget_bytes: int, k_max: int, opts=None):
    """Returns (status, server handle)."""
    h = ctypes.c_void_p()
    status = lib().di_serve_create(int(hbm_budget_bytes), int(k_max),
                                   ctypes.byref(opts) if opts is not None else None, ctypes.byref(h))
    return status, h


def di_serve_add_graph(s, g, graph_id: int) -> int:
    return lib().di_serve_add_graph(s, g, int(graph_id))


def di_serve_submit(s, graph_id: int, seeds, d: float, tol: float):
    """seeds: int32 ids (empty or None = uniform B). Returns (status, ticket)."""
    seeds = np.ascontiguousarray(np.asarray([] if seeds is None else seeds, dtype=np.int32))
    t = ctypes.c_uint64(0)
    status = lib().di_serve_submit(s, int(graph_id), int(seeds.size),
                                   seeds.ctypes.data if seeds.size else None, float(d), float(tol),
                                   ctypes.byref(t))
    return status, t.value


def di_serve_poll(s, ticket: int, X=None):
    """X: float64 host array of n values (or None). Returns (status, stats)."""
    st = di_stats()
    status = lib().di_serve_poll(s, ctypes.c_uint64(ticket), _ptr(X), ctypes.byref(st))
    return status, st


def di_serve_info(s):
    out = di_serve_stats()
    status = lib().di_serve_info(s, ctypes.byref(out))
    return status, out


def di_serve_destroy(s) -> None:
    lib().di_serve_destroy(s)


def _tol_array(tol, k: int):
    t = np.ascontiguousarray(np.asarray(tol, np.float64).ravel())
    if t.size == 1 and k > 1:
        t = np.full(k, t[0])
    return t


def _graph_n(h) -> int:
    n = ctypes.c_int64()
    _check(lib().di_graph_info(h, ctypes.byref(n), None, None, None))
    return n.value


class Graph:
    """Owning wrapper of a di_graph handle."""

    def __init__(self, n: int, src, dst):
        status, h = di_graph_create(n, src, dst)
        _check(status)
        self.handle = h
        self.n, self.L, self.n_dangling, self.n_loops = di_graph_info(h)

    def close(self):
        if getattr(self, "handle", None):
            di_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(g: Graph, B=None, d: float = 0.85, tol: float = 1e-9, **opt_fields):
    """Host convenience: returns (X as float64 numpy array, stats dict).
    Raises DIError unless the status is DI_OK."""
    o = di_opts_default()
    for k, v in opt_fields.items():
        setattr(o, k, v)
    X = np.empty(g.n, dtype=np.float64)
    Bh = None if B is None else np.ascontiguousarray(B, dtype=np.float64)
    status, st = di_solve(g.handle, Bh, d, tol, o, X)
    _check(status)
    return X, st.as_dict()
