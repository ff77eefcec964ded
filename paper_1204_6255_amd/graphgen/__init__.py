"""Seeded synthetic web-like digraphs and their Table-1 statistics.

Inputs only: nothing here computes any part of the D-iteration. The native
generator lives in ``graphgen.cpp`` (built into ``libdigen.so`` next to this
file); the recipe is described at the top of that file.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdigen.so")
_lib = None

# Parameters of the two generator readings of the web-graph recipe.
ALPHA_L_MATCHED = 1.68  # edge volume of about 7.6 links per node at kmax 500
ALPHA_LITERAL = 2.1


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("alpha", ctypes.c_double),
        ("kmax", ctypes.c_int32),
        ("radius", ctypes.c_int32),
        ("p_dangling", ctypes.c_double),
        ("p_local", ctypes.c_double),
        ("p_forward", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("L", ctypes.c_int64),
        ("D", ctypes.c_int64),
        ("zero_in", ctypes.c_int64),
        ("E", ctypes.c_int64),
        ("O", ctypes.c_int64),
        ("max_in", ctypes.c_int64),
        ("max_out", ctypes.c_int64),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(
            f"{_LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')"
        )
    lib = ctypes.CDLL(_LIB_PATH)
    lib.dg_generate.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
    lib.dg_generate.restype = ctypes.c_int
    lib.dg_num_edges.argtypes = [ctypes.c_void_p]
    lib.dg_num_edges.restype = ctypes.c_int64
    lib.dg_copy_edges.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.dg_copy_edges.restype = None
    lib.dg_free.argtypes = [ctypes.c_void_p]
    lib.dg_free.restype = None
    lib.dg_graph_stats.argtypes = [
        ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Stats)
    ]
    lib.dg_graph_stats.restype = ctypes.c_int
    _lib = lib
    return lib


def web_graph(n: int, seed: int = 0, alpha: float = ALPHA_L_MATCHED, kmax: int = 500,
              p_dangling: float = 0.15, p_local: float = 0.7, radius: int = 500,
              p_forward: float = 0.0):
    """Return (src, dst) int32 arrays of a synthetic web-like digraph.

    Links are sorted by (src, dst), without self-loops or duplicates.
    p_forward > 0 turns local links forward with that probability.
    """
    lib = _load()
    p = _Params(int(n), int(seed) & ((1 << 64) - 1), float(alpha), int(kmax), int(radius),
                float(p_dangling), float(p_local), float(p_forward))
    h = ctypes.c_void_p()
    rc = lib.dg_generate(ctypes.byref(p), ctypes.byref(h))
    if rc != 0:
        raise ValueError(f"dg_generate failed with status {rc}")
    try:
        m = lib.dg_num_edges(h)
        src = np.empty(m, dtype=np.int32)
        dst = np.empty(m, dtype=np.int32)
        lib.dg_copy_edges(h, src.ctypes.data, dst.ctypes.data)
    finally:
        lib.dg_free(h)
    return src, dst


@dataclass
class GraphStats:
    n: int
    L: int
    D: int
    zero_in: int
    E: int
    O: int
    max_in: int
    max_out: int

    def table1_row(self) -> dict:
        """The columns of the paper's Table 1, per node where the table uses ratios."""
        n = max(self.n, 1)
        return {
            "N": self.n, "L/N": self.L / n, "D/N": self.D / n, "E/N": self.E / n,
            "O/N": self.O / n, "max_in": self.max_in, "max_out": self.max_out,
            "zero_in/N": self.zero_in / n,
        }


def graph_stats(n: int, src, dst) -> GraphStats:
    """L, D, E, O, max_in, max_out (Section 2.4) of a link list."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    st = _Stats()
    rc = lib.dg_graph_stats(int(n), int(src.size), src.ctypes.data, dst.ctypes.data, ctypes.byref(st))
    if rc != 0:
        raise ValueError(f"dg_graph_stats failed with status {rc}")
    return GraphStats(st.n, st.L, st.D, st.zero_in, st.E, st.O, st.max_in, st.max_out)


def uniform_rhs(n: int, d: float) -> np.ndarray:
    """B = (1-d)/N for every node (the PageRank right-hand side)."""
    return np.full(n, (1.0 - d) / n, dtype=np.float64)


def ppr_seed_sets(n: int, k: int, base_seed: int = 1000, max_size: int = 100):
    """k seed sets for personalized PageRank: set j has a size uniform in
    [1, max_size] and its nodes are drawn without replacement, seeded by
    base_seed + j."""
    sets = []
    for j in range(k):
        rng = np.random.default_rng(base_seed + j)
        size = int(rng.integers(1, min(max_size, n) + 1))
        sets.append(np.sort(rng.choice(n, size=size, replace=False)).astype(np.int32))
    return sets


def ppr_rhs(n: int, seeds, d: float) -> np.ndarray:
    """B = (1-d)/|S| on the seed set S, zero elsewhere (sums to 1-d)."""
    b = np.zeros(n, dtype=np.float64)
    seeds = np.asarray(seeds)
    b[seeds] = (1.0 - d) / seeds.size
    return b


def random_small_graph(n: int, p_edge: float, rng, self_loops: bool = True):
    """Small random digraph for brute-force checks: each ordered pair (i, j)
    is a link with probability p_edge (i == j only if self_loops).
    Returned sorted by (src, dst)."""
    mask = rng.random((n, n)) < p_edge
    if not self_loops:
        np.fill_diagonal(mask, False)
    src, dst = np.nonzero(mask)
    return src.astype(np.int32), dst.astype(np.int32)


def transpose(src, dst):
    """The transposed link list (every link j -> i becomes i -> j), sorted
    by (origin, destination): the workload of P's transpose, where the
    generator's in-degree hubs become out-degree hubs."""
    s = np.ascontiguousarray(dst, dtype=np.int32)
    t = np.ascontiguousarray(src, dtype=np.int32)
    order = np.lexsort((t, s))
    return s[order], t[order]


def prefix_subgraph(m: int, src, dst):
    """The subgraph induced on the node ids [0, m): the links with both ends
    below m, in the original (sorted) order."""
    src = np.asarray(src)
    dst = np.asarray(dst)
    keep = (src < m) & (dst < m)
    return (np.ascontiguousarray(src[keep], dtype=np.int32),
            np.ascontiguousarray(dst[keep], dtype=np.int32))
