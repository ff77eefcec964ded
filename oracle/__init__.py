"""Plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It wraps ``oracle.c`` (built into ``liboracle.so``)
through ctypes; the C file states the definitions and readings it follows.

Functions (all FP64, single thread):
  Graph(n, src, dst)              the l_out / l_in iterators of Section 2.1
  diter(g, B, d, ...)             DI-SOP / DI-CYC (Sections 2.5.4-2.5.5), in the
                                  paper's sequential cycle or the labelled
                                  SYNC and TILED schedules of the GPU
  di_cycle(g, F, H, ...)          one D-iteration cycle, in place
  pi(g, d, ...)                   PI / PI' (Sections 2.5.1-2.5.2)
  jacobi(g, B, d, tol)            unnormalized power (Jacobi) iteration
  gs(g, B, d, ...)                Gauss-Seidel (Section 2.5.3)
  residual(g, B, d, X)            R = B + P.X - X and ||R||_1
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DI_ORACLE_LIB names another build of oracle.c (the sanitizer test's)
_LIB_PATH = os.environ.get("DI_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

SOP, CYC = 0, 1
SEQUENTIAL, SYNC, TILED = 0, 1, 2
STOP_RESID, STOP_PAPER = 0, 1

OK, E_INVAL, E_DUP, E_RANGE, E_NOMEM, E_NOCONV = 0, -1, -3, -4, -5, -6


class _Stats(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int64),
        ("link_ops", ctypes.c_int64),
        ("fallback_cycles", ctypes.c_int64),
        ("nb_iter", ctypes.c_double),
        ("resid_l1", ctypes.c_double),
        ("paper_err", ctypes.c_double),
        ("e", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


@dataclass
class Stats:
    status: int
    cycles: int
    link_ops: int
    fallback_cycles: int
    nb_iter: float
    resid_l1: float
    paper_err: float
    e: float
    seconds: float


def _stats(rc, s: _Stats) -> Stats:
    return Stats(rc, s.cycles, s.link_ops, s.fallback_cycles, s.nb_iter, s.resid_l1,
                 s.paper_err, s.e, s.seconds)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: run oracle/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.orc_graph_build.argtypes = [i64, i64, vp, vp, ctypes.POINTER(vp)]
    lib.orc_graph_build.restype = i32
    lib.orc_graph_free.argtypes = [vp]
    lib.orc_graph_free.restype = None
    lib.orc_residual.argtypes = [vp, vp, dbl, vp, vp]
    lib.orc_residual.restype = dbl
    lib.orc_apply_p.argtypes = [vp, dbl, vp, vp]
    lib.orc_apply_p.restype = None
    lib.orc_di_cycle.argtypes = [vp, dbl, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_di_cycle.restype = i64
    lib.orc_diter.argtypes = [vp, vp, dbl, i32, i32, i32, dbl, i64, vp, vp, ctypes.POINTER(_Stats)]
    lib.orc_diter.restype = i32
    lib.orc_di_cycle2.argtypes = [vp, dbl, i32, i32, i64, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_di_cycle2.restype = i64
    lib.orc_diter2.argtypes = [vp, vp, dbl, i32, i32, i64, i64, i32, i32, dbl, i64, vp, vp,
                               ctypes.POINTER(_Stats)]
    lib.orc_diter2.restype = i32
    lib.orc_pi.argtypes = [vp, dbl, i32, dbl, i64, vp, ctypes.POINTER(_Stats)]
    lib.orc_pi.restype = i32
    lib.orc_jacobi.argtypes = [vp, vp, dbl, dbl, i64, vp, ctypes.POINTER(_Stats)]
    lib.orc_jacobi.restype = i32
    lib.orc_gs.argtypes = [vp, vp, dbl, i32, dbl, i64, vp, ctypes.POINTER(_Stats)]
    lib.orc_gs.restype = i32
    _lib = lib
    return lib


def _f64(a, n):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


class Graph:
    """P built from a link list (origin src[e] -> destination dst[e])."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        self.n = int(n)
        self._src = np.ascontiguousarray(src, dtype=np.int32)
        self._dst = np.ascontiguousarray(dst, dtype=np.int32)
        if self._src.shape != self._dst.shape:
            raise ValueError("src and dst differ in length")
        self.L = int(self._src.size)
        h = ctypes.c_void_p()
        rc = lib.orc_graph_build(self.n, self.L, self._src.ctypes.data, self._dst.ctypes.data,
                                 ctypes.byref(h))
        if rc != OK:
            raise ValueError(f"orc_graph_build failed with status {rc}")
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_graph_free(h)
            self._h = None


def residual(g: Graph, B, d: float, X):
    """(R, ||R||_1) with R = B + P.X - X."""
    lib = _load()
    B = _f64(B, g.n)
    X = _f64(X, g.n)
    R = np.empty(g.n)
    l1 = lib.orc_residual(g.handle, B.ctypes.data, d, X.ctypes.data, R.ctypes.data)
    return R, l1


def apply_p(g: Graph, d: float, x):
    lib = _load()
    x = _f64(x, g.n)
    y = np.empty(g.n)
    lib.orc_apply_p(g.handle, d, x.ctypes.data, y.ctypes.data)
    return y


def diter(g: Graph, B, d: float, variant: int = SOP, schedule: int = SEQUENTIAL,
          stop: int = STOP_RESID, tol: float = 1e-9, max_cycles: int = 1_000_000,
          tile: int = 1, reach: int = 0, rounds: int = 1):
    """D-iteration solve. Returns (H, F, Stats); H approximates X.
    schedule TILED takes tile, reach and rounds (see di_cycle)."""
    lib = _load()
    B = _f64(B, g.n)
    H = np.empty(g.n)
    F = np.empty(g.n)
    st = _Stats()
    rc = lib.orc_diter2(g.handle, B.ctypes.data, d, variant, schedule, tile, reach, rounds, stop,
                        tol, max_cycles, H.ctypes.data, F.ctypes.data, ctypes.byref(st))
    if rc not in (OK, E_NOCONV):
        raise ValueError(f"orc_diter failed with status {rc}")
    return H, F, _stats(rc, st)


def di_cycle(g: Graph, F, H, d: float, variant: int = SOP, schedule: int = SEQUENTIAL, e: float = 0.0,
             tile: int = 1, reach: int = 0, rounds: int = 1):
    """One cycle in place on float64 arrays F, H.
    Returns (count, selected mask, e, link_ops, r used).
    schedule TILED: `rounds` frontier-synchronous rounds per cycle (DI-SOP;
    DI-CYC runs one) over tiles of `tile` ids; an amount sent along i -> j
    with |i - j| <= reach inside i's tile is seen by the later rounds, any
    other waits for the next cycle. count counts diffusions over the rounds."""
    lib = _load()
    if F.dtype != np.float64 or H.dtype != np.float64 or not F.flags.c_contiguous or not H.flags.c_contiguous:
        raise ValueError("F and H must be contiguous float64 arrays")
    if schedule == TILED and (tile < 1 or reach < 0 or rounds < 1):
        raise ValueError("TILED needs tile >= 1, reach >= 0, rounds >= 1")
    sel = np.zeros(g.n, dtype=np.uint8)
    claim = np.empty(max(g.n, 1))
    nxt = np.empty(max(g.n, 1))
    e_c = ctypes.c_double(e)
    ops = ctypes.c_int64(0)
    r = ctypes.c_double(0.0)
    cnt = lib.orc_di_cycle2(g.handle, d, variant, schedule, tile, reach, rounds, F.ctypes.data,
                            H.ctypes.data, ctypes.byref(e_c), ctypes.byref(ops), sel.ctypes.data,
                            claim.ctypes.data, nxt.ctypes.data, ctypes.byref(r))
    return int(cnt), sel.astype(bool), e_c.value, ops.value, r.value


def pi(g: Graph, d: float, by_columns: bool = False, target: float | None = None,
       max_iter: int = 100_000):
    """PI (rows) or PI' (columns), normalized; target defaults to 1/N."""
    lib = _load()
    x = np.empty(g.n)
    st = _Stats()
    t = 1.0 / g.n if target is None else target
    rc = lib.orc_pi(g.handle, d, 1 if by_columns else 0, t, max_iter, x.ctypes.data, ctypes.byref(st))
    if rc not in (OK, E_NOCONV):
        raise ValueError(f"orc_pi failed with status {rc}")
    return x, _stats(rc, st)


def jacobi(g: Graph, B, d: float, tol: float = 1e-9, max_iter: int = 100_000):
    lib = _load()
    B = _f64(B, g.n)
    x = np.empty(g.n)
    st = _Stats()
    rc = lib.orc_jacobi(g.handle, B.ctypes.data, d, tol, max_iter, x.ctypes.data, ctypes.byref(st))
    if rc not in (OK, E_NOCONV):
        raise ValueError(f"orc_jacobi failed with status {rc}")
    return x, _stats(rc, st)


def gs(g: Graph, B, d: float, stop: int = STOP_RESID, tol: float = 1e-9, max_sweeps: int = 100_000):
    lib = _load()
    B = _f64(B, g.n)
    x = np.empty(g.n)
    st = _Stats()
    rc = lib.orc_gs(g.handle, B.ctypes.data, d, stop, tol, max_sweeps, x.ctypes.data, ctypes.byref(st))
    if rc not in (OK, E_NOCONV):
        raise ValueError(f"orc_gs failed with status {rc}")
    return x, _stats(rc, st)
