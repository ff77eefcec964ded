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


def _powerlaw_exponent(mean: float, kmax: int) -> float:
    """The exponent a of P(k) proportional to k^-a on [1, kmax] whose mean is
    `mean` (bisection; the mean falls as a grows)."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    lo, hi = 0.0, 8.0
    for _ in range(80):
        a = 0.5 * (lo + hi)
        p = k ** -a
        if (k * p).sum() / p.sum() > mean:
            lo = a
        else:
            hi = a
    return 0.5 * (lo + hi)


def high_e_graph(n: int = 9664, seed: int = 0, e_frac: float = 0.91, d_frac: float = 0.48,
                 links_per_node: float = 1.67, kmax: int = 164, kernel_frac: float = 0.01,
                 p_core: float = 0.3, p_back: float = 0.05, beta: float = 0.6):
    """A web-like digraph where most nodes are 0 in-degree nodes in the
    recursive sense of Section 2.4 (E): the stand-in for the gr0.California
    graph of Section 2.8, whose Table 9 gives L/N 1.67, D/N 0.48, E/N 0.91,
    O/N 0, max_in 199, max_out 164 at N = 9664.

    Construction (node positions, shuffled into ids at the end):
    - the non-E part, (1 - e_frac)·n nodes: a kernel of kernel_frac·n nodes
      joined in a ring (so every kernel node lies on a cycle), followed by a
      tail in which every node has a parent link from an earlier non-E node
      that is not dangling (so it lies downstream of the ring); kernel nodes
      link inside the non-E part, tail nodes link forward in the tail or,
      with probability p_back, back into the kernel;
    - the E part, e_frac·n nodes in a topological order: each links forward
      inside the E part or, with probability p_core, into the non-E part.
      Nothing links into the E part from outside it, so its nodes are
      exactly the recursive 0 in-degree nodes;
    - d_frac·n dangling nodes drawn among the E part and the tail; the other
      nodes draw an out-degree from a power law on [1, kmax] whose mean
      gives links_per_node·n links (the ring and parent links count in it);
    - each link's destination is drawn among its allowed positions with
      weight rank^-beta (ranks a seeded permutation), which makes in-degree
      hubs.
    No self-loops or duplicate links. Sorted by (src, dst), int32.
    """
    if n < 4:
        raise ValueError("high_e_graph needs n >= 4")
    rng = np.random.default_rng(seed)
    n_core = max(2, int(round((1.0 - e_frac) * n)))
    n_ker = max(2, min(n_core, int(round(kernel_frac * n))))
    n_e = n - n_core
    k0, t0 = n_e, n_e + n_ker  # kernel [k0, t0), tail [t0, n)
    cand = np.concatenate([np.arange(n_e), np.arange(t0, n)])
    dang = np.zeros(n, dtype=bool)
    dang[rng.choice(cand, size=min(int(round(d_frac * n)), cand.size), replace=False)] = True
    active = np.flatnonzero(~dang)
    forced = {v: {k0 + (v - k0 + 1) % n_ker} for v in range(k0, t0)}
    feeders = np.flatnonzero(~dang[k0:]) + k0  # ascending; the kernel comes first
    for u in range(t0, n):
        c = int(feeders[int(rng.integers(int(np.searchsorted(feeders, u))))])
        forced.setdefault(c, set()).add(u)
    n_forced = np.zeros(n, dtype=np.int64)
    for v, f in forced.items():
        n_forced[v] = len(f)
    a = _powerlaw_exponent(links_per_node * n / active.size, kmax)
    pk = np.arange(1, kmax + 1, dtype=np.float64) ** -a
    cdf = np.cumsum(pk) / pk.sum()
    out_deg = np.zeros(n, dtype=np.int64)
    out_deg[active] = np.minimum(1 + np.searchsorted(cdf, rng.random(active.size), side="right"),
                                 kmax)
    out_deg = np.maximum(out_deg, n_forced)
    # the sum of a heavy-tailed draw strays from its mean: move single links
    # between random nodes until the total is the target
    excess = int(out_deg.sum()) - int(round(links_per_node * n))
    floor = np.maximum(n_forced, 1)
    excess = max(min(excess, int((out_deg - floor)[active].sum())),
                 -int((kmax - out_deg)[active].clip(min=0).sum()))
    while excess != 0:
        v = int(active[int(rng.integers(active.size))])
        if excess > 0 and out_deg[v] > floor[v]:
            out_deg[v] -= 1
            excess -= 1
        elif excess < 0 and out_deg[v] < kmax:
            out_deg[v] += 1
            excess += 1
    cw = np.concatenate([[0.0], np.cumsum((rng.permutation(n) + 1.0) ** -beta)])

    def pick(lo, hi):
        u = cw[lo] + rng.random() * (cw[hi] - cw[lo])
        return min(max(int(np.searchsorted(cw, u, side="right")) - 1, lo), hi - 1)

    links = set()
    for v in active.tolist():
        got = set(forced.get(v, ()))
        if k0 <= v < t0:
            ranges = [(k0, n, 1.0)]
        elif v < n_e:
            ranges = [(v + 1, n_e, 1.0 - p_core), (k0, n, p_core)]
        else:
            ranges = [(v + 1, n, 1.0 - p_back), (k0, t0, p_back)]
        ranges = [r for r in ranges if r[1] > r[0]]
        room = sum(hi - lo for lo, hi, _ in ranges) - (1 if any(lo <= v < hi for lo, hi, _ in ranges)
                                                       else 0)
        cap = max(min(int(out_deg[v]), room), len(got))
        total = sum(p for _, _, p in ranges)
        tries = 0
        while len(got) < cap and tries < 20 * cap:
            tries += 1
            x = rng.random() * total
            for lo, hi, p in ranges:
                if x < p:
                    break
                x -= p
            t = pick(lo, hi)
            if t != v:
                got.add(t)
        links.update((v, t) for t in got)
    arr = np.array(sorted(links), dtype=np.int64).reshape(-1, 2)
    perm = rng.permutation(n)
    s, t = perm[arr[:, 0]], perm[arr[:, 1]]
    order = np.lexsort((t, s))
    return s[order].astype(np.int32), t[order].astype(np.int32)
