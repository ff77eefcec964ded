"""GPU parity of the FP64 residual pass and of FP32 solves with FP64
refinement (DI_FP32_REFINE) against the CPU oracle.

The residual pass is compared entry by entry with the oracle's R = B + P.X
- X, within a rounding bound derived from the magnitudes that enter each
entry. A refined solve must return an X whose residual, recomputed by the
oracle, is within tol, and whose distance to the oracle's X is within the
error bound tol / (1 - d) (P's columns sum to at most d) plus the oracle's
own 1e-13.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen

pytestmark = pytest.mark.gpu

D = 0.85
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


_GRAPHS = {}


def web(n, alpha=graphgen.ALPHA_L_MATCHED, seed=0):
    key = (n, alpha, seed)
    if key not in _GRAPHS:
        _GRAPHS[key] = graphgen.web_graph(n, seed=seed, alpha=alpha)
    return _GRAPHS[key]


def star(n):
    """Node 0 links to every other node and every other node links to 0:
    one row with n - 1 in-links (split into segments by the pull)."""
    src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)]).astype(np.int32)
    dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)]).astype(np.int32)
    order = np.lexsort((dst, src))
    return src[order], dst[order]


def with_self_loops(n, src, dst, every=7):
    """Adds a self-loop to every `every`-th node (sorted, no duplicates)."""
    keep = src != dst
    s = np.concatenate([src[keep], np.arange(0, n, every, dtype=np.int32)])
    t = np.concatenate([dst[keep], np.arange(0, n, every, dtype=np.int32)])
    order = np.lexsort((t, s))
    return s[order].astype(np.int32), t[order].astype(np.int32)


def residual_gpu(torch, g, B, X):
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float64)).cuda()
    Bd = None if B is None else torch.from_numpy(np.ascontiguousarray(B, np.float64)).cuda()
    R = torch.empty(g.n, dtype=torch.float64, device="cuda")
    status, l1 = di.di_residual_dev(g.handle, Bd, D, Xd, R)
    assert status == di.DI_OK, di.di_last_error()
    torch.cuda.synchronize()
    return R.cpu().numpy(), l1


def check_residual(torch, n, src, dst, B, X):
    og = oracle.Graph(n, src, dst)
    Bfull = graphgen.uniform_rhs(n, D) if B is None else B
    R_ref, l1_ref = oracle.residual(og, Bfull, D, X)
    R, l1 = residual_gpu(torch, di.Graph(n, src, dst), B, X)
    # every entry: B_i - X_i + sum of d X_j / out_j; the sums differ only in
    # their rounding order, so the gap is bounded by a few ulps of the
    # magnitudes involved
    scale = np.abs(Bfull) + np.abs(X) + oracle.apply_p(og, D, np.abs(X))
    bound = 4 * (np.log2(max(og.n, 2)) + 8) * EPS * scale
    assert np.all(np.abs(R - R_ref) <= bound), np.max(np.abs(R - R_ref) / np.maximum(bound, 1e-300))
    assert abs(l1 - l1_ref) <= bound.sum() + 4 * n * EPS * l1_ref


@pytest.mark.parametrize("case", ["web10k", "web10k_literal", "loops", "star"])
def test_residual_pass_entrywise(torch_cuda, case):
    rng = np.random.default_rng(5)
    if case == "star":
        n = 30001
        src, dst = star(n)
    else:
        n = 10000
        src, dst = web(n, alpha=graphgen.ALPHA_LITERAL if case == "web10k_literal"
                       else graphgen.ALPHA_L_MATCHED)
        if case == "loops":
            src, dst = with_self_loops(n, src, dst)
    X = rng.random(n) / n
    check_residual(torch_cuda, n, src, dst, None, X)
    B = rng.standard_normal(n) * 1e-4
    check_residual(torch_cuda, n, src, dst, B, X)


def test_residual_pass_1m_at_the_solution(torch_cuda):
    """At the oracle's solution of the benchmark graph the residual is a
    sum of cancelling terms; it must still match entry by entry."""
    n = 1_000_000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    X_ref, _, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-11)
    check_residual(torch_cuda, n, src, dst, None, X_ref)


def refined(torch, g, B, tol, allow=(di.DI_OK,), **fields):
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    for k, v in fields.items():
        setattr(o, k, v)
    X = torch.empty(g.n, dtype=torch.float64, device="cuda")
    Bd = None if B is None else torch.from_numpy(np.ascontiguousarray(B, np.float64)).cuda()
    status, st = di.di_solve_dev(g.handle, Bd, D, tol, o, X)
    assert status in allow, (di.STATUS_NAMES.get(status), di.di_last_error())
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, status


def oracle_solution(og, B):
    H, _, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert st.status == oracle.OK
    return H


@pytest.mark.parametrize("kernel", [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW])
@pytest.mark.parametrize("rhs", ["uniform", "ppr", "signed"])
def test_refined_solve_10k(torch_cuda, kernel, rhs):
    n = 10000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    if rhs == "uniform":
        B, Bd = graphgen.uniform_rhs(n, D), None
    elif rhs == "ppr":
        B = graphgen.ppr_rhs(n, graphgen.ppr_seed_sets(n, 1)[0], D)
        Bd = B
    else:
        B = np.random.default_rng(3).standard_normal(n) * 1e-4
        Bd = B
    X_ref = oracle_solution(og, B)
    tol = 1.4e-10
    X, st, _ = refined(torch_cuda, di.Graph(n, src, dst), Bd, tol, kernel=kernel)
    _, r_true = oracle.residual(og, B, D, X)
    assert st.refinements >= 1
    assert st.resid_l1 <= tol
    assert abs(r_true - st.resid_l1) <= 1e-15 + 1e-6 * st.resid_l1
    assert np.abs(X - X_ref).sum() <= tol / (1 - D) + 1e-12


def test_refined_solve_1m_bench_configuration(torch_cuda):
    n = 1_000_000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    X_ref = oracle_solution(og, B)
    g = di.Graph(n, src, dst)
    X, st, _ = refined(torch_cuda, g, None, 1e-9)
    _, r_true = oracle.residual(og, B, D, X)
    assert st.resid_l1 <= 1e-9 and r_true <= 1e-9 * (1 + 1e-6)
    assert np.abs(X - X_ref).sum() <= st.err_bound + 1e-12
    assert 1 <= st.refinements <= 4
    # a tighter inner target needs no more refinements
    X2, st2, _ = refined(torch_cuda, g, None, 1e-9, inner_tol=1e-7)
    assert st2.resid_l1 <= 1e-9 and st2.refinements <= st.refinements


def test_refined_signed_1m_window(torch_cuda):
    """A signed right-hand side at N = 1M on the window push: the FP32
    passes take r from the records' bound of sum |F| (no gathering after
    each cycle), and the FP64 residual passes still decide convergence: the
    residual the oracle recomputes is within tol and X within tol / (1 - d)
    of the oracle's."""
    n = 1_000_000
    src, dst = web(n)
    og = oracle.Graph(n, src, dst)
    B = np.random.default_rng(11).standard_normal(n) * (1.0 / n)
    print("refined signed 1M: oracle solve", flush=True)
    X_ref = oracle_solution(og, B)
    g = di.Graph(n, src, dst)
    print("refined signed 1M: GPU solve", flush=True)
    tol = 1e-9
    X, st, _ = refined(torch_cuda, g, B, tol, kernel=di.DI_KERNEL_WINDOW)
    _, r_true = oracle.residual(og, B, D, X)
    assert st.refinements >= 1
    assert st.resid_l1 <= tol and r_true <= tol * (1 + 1e-6)
    assert abs(r_true - st.resid_l1) <= 1e-15 + 1e-6 * st.resid_l1
    assert np.abs(X - X_ref).sum() <= tol / (1 - D) + 1e-12


def test_refined_edge_cases(torch_cuda):
    torch = torch_cuda
    # one node, no links: X = B / 1 after one pass
    g1 = di.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    X, st, _ = refined(torch, g1, None, 1e-12)
    assert abs(X[0] - (1 - D)) <= 1e-15
    # B = 0: converged before any cycle, X = 0
    n = 2000
    src, dst = web(n)
    g = di.Graph(n, src, dst)
    X, st, _ = refined(torch, g, np.zeros(n), 1e-9)
    assert st.cycles == 0 and st.refinements == 0 and not X.any()
    # max_cycles: NOCONV, X still holds the folded history
    X, st, status = refined(torch, g, None, 1e-14, allow=(di.DI_E_NOCONV,), max_cycles=5)
    assert status == di.DI_E_NOCONV and st.cycles == 5 and st.refinements >= 1
    og = oracle.Graph(n, src, dst)
    _, r_true = oracle.residual(og, graphgen.uniform_rhs(n, D), D, X)
    assert abs(r_true - st.resid_l1) <= 1e-15 + 1e-6 * r_true
    # the paper's stopping rule has no meaning for a refined solve
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    o.stop = di.DI_STOP_PAPER
    Xd = torch.empty(n, dtype=torch.float64, device="cuda")
    status, _ = di.di_solve_dev(g.handle, None, D, 1.0 / n, o, Xd)
    assert status == di.DI_E_INVAL
    # residual entry point: NULL X is rejected, NULL R gives the norm only
    status, _ = di.di_residual_dev(g.handle, None, D, None)
    assert status == di.DI_E_INVAL
    Xr = torch.from_numpy(oracle_solution(og, graphgen.uniform_rhs(n, D))).cuda()
    status, l1 = di.di_residual_dev(g.handle, None, D, Xr)
    assert status == di.DI_OK and l1 <= 1e-12
