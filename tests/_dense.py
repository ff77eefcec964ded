"""Dense linear algebra used to pin the oracle (small graphs only).

P is built straight from the link list: P[i, j] = d / out_j for each link
j -> i, so X = solve(I - P, B) is the definition of the solution.
"""

import numpy as np


def dense_p(n, src, dst, d):
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    out = np.bincount(src, minlength=n).astype(np.float64)
    P = np.zeros((n, n))
    for j, i in zip(src, dst):
        P[i, j] += d / out[j]
    return P


def dense_solve(n, src, dst, d, B):
    P = dense_p(n, src, dst, d)
    return np.linalg.solve(np.eye(n) - P, np.asarray(B, dtype=np.float64)), P
