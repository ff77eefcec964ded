"""GPU parity of batched solves (k right-hand sides on one graph) against
the CPU oracle, one oracle solve per column.

Reading: each column is its own DI-SOP solve, so column c must satisfy
|X_c - X_ref_c|_1 <= tol_c / (1 - d) (the columns of P sum to at most d, so
|(I - P)^-1|_1 <= 1 / (1 - d) bounds the error by the residual) plus
the oracle's own 1e-13, and its residual recomputed by the oracle must be
within tol_c. Columns with the same right-hand side in one batch go through
the same arithmetic and must agree bit for bit.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen

pytestmark = pytest.mark.gpu

D = 0.85

_GRAPHS = {}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def web(n, alpha=graphgen.ALPHA_L_MATCHED, seed=0):
    key = (n, alpha, seed)
    if key not in _GRAPHS:
        _GRAPHS[key] = graphgen.web_graph(n, seed=seed, alpha=alpha)
    return _GRAPHS[key]


def ppr_matrix(n, k, base_seed=1000):
    return np.stack([graphgen.ppr_rhs(n, s, D) for s in graphgen.ppr_seed_sets(n, k, base_seed)])


def oracle_x(og, B):
    H, _, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert st.status == oracle.OK
    return H


def batch(g, k, B, tol, allow=(di.DI_OK,), **fields):
    o = di.di_opts_default()
    for name, v in fields.items():
        setattr(o, name, v)
    status, X, st = di.di_solve_batch(g.handle, k, B, D, tol, o)
    assert status in allow, (di.STATUS_NAMES.get(status), di.di_last_error())
    return X, st, status


def check_columns(og, B, X, st, tol, cols):
    for c in cols:
        Bc = B[c] if B is not None else graphgen.uniform_rhs(og.n, D)
        ref = oracle_x(og, Bc)
        _, r_true = oracle.residual(og, Bc, D, X[c])
        assert r_true <= tol[c] * (1 + 1e-6) + 1e-16, (c, r_true, tol[c])
        assert st[c].resid_l1 <= tol[c]
        assert np.abs(X[c] - ref).sum() <= tol[c] / (1 - D) + 1e-12, c


@pytest.mark.parametrize("precision", [di.DI_FP64, di.DI_FP32_REFINE])
@pytest.mark.parametrize("k", [1, 5, 8, 13, 40])
def test_batch_10k_vs_oracle(torch_cuda, precision, k):
    n = 10000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    B = ppr_matrix(n, k)
    # mixed tolerances: 1e-9 and 1e-6 alternate (per-column stop)
    tol = np.where(np.arange(k) % 2 == 0, 1e-9, 1e-6) * (1 - D)
    X, st, _ = batch(di.Graph(n, src, dst), k, B, tol, precision=precision)
    check_columns(og, B, X, st, tol, range(k))
    if precision == di.DI_FP32_REFINE:
        assert all(s.refinements >= 1 for s in st)


def test_batch_column_independence(torch_cuda):
    """The same right-hand side twice in a batch: identical columns; a
    column alone and inside a larger batch: the same solution."""
    n = 10000
    src, dst = web(n)
    g = di.Graph(n, src, dst)
    B = ppr_matrix(n, 20)
    B[7] = B[3]
    B[19] = B[3]
    tol = np.full(20, 1e-10)
    X, st, _ = batch(g, 20, B, tol)
    assert np.array_equal(X[7], X[3]) and np.array_equal(X[19], X[3])
    assert st[7].cycles == st[3].cycles and st[7].edges_pushed == st[3].edges_pushed
    # alone (another lane layout, so other rounding): the same solution
    # within the error bounds of the two solves
    X1, st1, _ = batch(g, 1, B[3:4], tol[:1])
    assert np.abs(X1[0] - X[3]).sum() <= 2 * 1e-10 / (1 - D)
    assert abs(st1[0].cycles - st[3].cycles) <= 1
    # and the single-RHS path agrees (the pull: the batch's frontier-
    # synchronous schedule, so the same cycles)
    Xs, sts = di.solve(g, B[3], D, 1e-10, kernel=di.DI_KERNEL_PULL)
    assert np.abs(Xs - X[3]).sum() <= 2 * 1e-10 / (1 - D)
    assert abs(sts["cycles"] - st[3].cycles) <= 1


@pytest.mark.parametrize("case", ["loops", "star", "literal"])
def test_batch_graph_shapes(torch_cuda, case):
    """Self-loops, a hub with 30000 in-links (split into pull segments), and
    the literal-exponent generator."""
    if case == "star":
        n = 30001
        src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)]).astype(np.int32)
        dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)]).astype(np.int32)
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
    else:
        n = 10000
        src, dst = web(n, alpha=graphgen.ALPHA_LITERAL if case == "literal" else graphgen.ALPHA_L_MATCHED)
        if case == "loops":
            keep = src != dst
            s = np.concatenate([src[keep], np.arange(0, n, 5, dtype=np.int32)])
            t = np.concatenate([dst[keep], np.arange(0, n, 5, dtype=np.int32)])
            order = np.lexsort((t, s))
            src, dst = s[order].astype(np.int32), t[order].astype(np.int32)
    og = oracle.Graph(n, src, dst)
    k = 16
    B = ppr_matrix(n, k, base_seed=7)
    B[0] = graphgen.uniform_rhs(n, D)
    tol = np.full(k, 1.4e-10)
    g = di.Graph(n, src, dst)
    for precision in (di.DI_FP64, di.DI_FP32_REFINE):
        X, st, _ = batch(g, k, B, tol, precision=precision)
        check_columns(og, B, X, st, tol, [0, 1, 9, 15])


def test_batch_1m_sampled_columns(torch_cuda):
    """The benchmark graph with 100 PPR columns (FP32 + FP64 refinement):
    every column within its tolerance, sampled columns against the oracle."""
    n = 1_000_000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    k = 100
    B = ppr_matrix(n, k)
    tol = np.full(k, 1e-9)
    X, st, _ = batch(di.Graph(n, src, dst), k, B, tol, precision=di.DI_FP32_REFINE)
    assert all(s.resid_l1 <= 1e-9 for s in st)
    check_columns(og, B, X, st, tol, [0, 57, 99])


def test_batch_device_entry_and_uniform_b(torch_cuda):
    torch = torch_cuda
    n = 5000
    src, dst = web(n, seed=3)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    k = 3
    Xd = torch.empty((k, n), dtype=torch.float64, device="cuda")
    tol = np.full(k, 1.4e-10)
    status, st = di.di_solve_batch_dev(g.handle, k, None, D, tol, None, Xd)
    assert status == di.DI_OK, di.di_last_error()
    torch.cuda.synchronize()
    X = Xd.cpu().numpy()
    ref = oracle_x(og, graphgen.uniform_rhs(n, D))
    for c in range(k):
        assert np.abs(X[c] - ref).sum() <= 1e-9
    assert np.array_equal(X[0], X[2])


def test_batch_edge_cases(torch_cuda):
    n = 2000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    B = ppr_matrix(n, 4)
    B[2] = 0.0  # converged before any cycle
    X, st, _ = batch(g, 4, B, np.full(4, 1e-10), precision=di.DI_FP32_REFINE)
    assert st[2].cycles == 0 and not X[2].any()
    check_columns(og, B, X, st, np.full(4, 1e-10), [0, 3])
    # more columns than one launch group holds (256 + 44), two groups
    k = 300
    Bk = ppr_matrix(n, k, base_seed=5)
    X, st, _ = batch(g, k, Bk, np.full(k, 1e-9))
    check_columns(og, Bk, X, st, np.full(k, 1e-9), [0, 255, 256, 299])
    # max_cycles: NOCONV for the columns that needed more
    X, st, status = batch(g, 4, ppr_matrix(n, 4), np.full(4, 1e-14), allow=(di.DI_E_NOCONV,),
                          max_cycles=3)
    assert status == di.DI_E_NOCONV and all(s.cycles == 3 for s in st)
    # invalid arguments
    o = di.di_opts_default()
    for k_bad in (0, -1):
        status, _, _ = di.di_solve_batch(g.handle, k_bad, None, D, [1e-9], o)
        assert status == di.DI_E_INVAL
    status, _, _ = di.di_solve_batch(g.handle, 2, None, D, [1e-9, 0.0], o)
    assert status == di.DI_E_INVAL
    Bn = ppr_matrix(n, 2)
    Bn[1, 5] = np.inf
    status, _, _ = di.di_solve_batch(g.handle, 2, Bn, D, [1e-9, 1e-9], o)
    assert status == di.DI_E_INVAL
    o.stop = di.DI_STOP_PAPER
    status, _, _ = di.di_solve_batch(g.handle, 1, None, D, [1e-9], o)
    assert status == di.DI_E_INVAL
    o = di.di_opts_default()
    o.kernel = di.DI_KERNEL_PUSH
    status, _, _ = di.di_solve_batch(g.handle, 1, None, D, [1e-9], o)
    assert status == di.DI_E_INVAL


def test_batch_k256_fp32_refine_at_1m(torch_cuda):
    """The widest batched shape of the benchmark: k = 256 personalized
    columns on the N = 1M graph in FP32 with FP64 residual passes (the float
    256-column kernels). Every column's residual, recomputed by the oracle,
    is within tol; eight columns (both ends of each 128-column half and four
    others) are within tol/(1-d) of oracle solves."""
    torch = torch_cuda
    n, k, tol = 1_000_000, 256, 1e-9
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    B = ppr_matrix(n, k)
    print(f"batch k={k} n={n} fp32+refine", flush=True)
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.empty((k, n), dtype=torch.float64, device="cuda")
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    status, st = di.di_solve_batch_dev(g.handle, k, Bd, D, np.full(k, tol), o, Xd)
    assert status == di.DI_OK, di.di_last_error()
    torch.cuda.synchronize()
    del Bd
    print("batch k=256: residuals", flush=True)
    for c in range(k):
        Xc = Xd[c].cpu().numpy()
        _, r = oracle.residual(og, B[c], D, Xc)
        assert r <= tol, (c, r)
        assert abs(r - st[c].resid_l1) <= 1e-14 + 1e-6 * tol, (c, r, st[c].resid_l1)
    print("batch k=256: oracle solves", flush=True)
    for c in (0, 1, 127, 128, 129, 200, 254, 255):
        ref = oracle_x(og, B[c])
        assert np.abs(Xd[c].cpu().numpy() - ref).sum() <= tol / (1 - D) + 1e-12, c
    g.close()
