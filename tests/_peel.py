"""The recursive 0 in-degree nodes of Section 2.4 (the E class) and their
depths, by peeling: a node joins once every one of its in-links comes from a
node that has joined (Kahn's topological order). Test host logic only."""

from collections import deque

import numpy as np


def e_depth(n, src, dst):
    """depth[i] = length of the longest path ending at i when i is an E node
    (0 for a node without in-links), -1 when i is not an E node (a cycle,
    self-loops included, lies upstream of it)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    indeg = np.bincount(dst, minlength=n)
    order = np.argsort(src, kind="stable")
    s, t = src[order], dst[order]
    start = np.searchsorted(s, np.arange(n + 1))
    depth = np.full(n, -1, dtype=np.int64)
    longest = np.zeros(n, dtype=np.int64)
    q = deque(np.flatnonzero(indeg == 0).tolist())
    left = indeg.copy()
    while q:
        v = q.popleft()
        depth[v] = longest[v]
        for w in t[start[v]:start[v + 1]].tolist():
            longest[w] = max(longest[w], longest[v] + 1)
            left[w] -= 1
            if left[w] == 0:
                q.append(w)
    return depth
