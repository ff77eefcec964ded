"""GPU parity on two more workloads of the paper's kind:

- the transposed web graph (Section 2.7, Dataset 1bis: the same graph
  with every link reversed), where the generator's in-degree hubs become
  nodes with tens of thousands of out-links;
- prefix subgraphs of the N = 1M graph (the subgraph induced on the node
  ids below m), the paper's way of varying N (Section 2.6, Table 1).

- a graph whose links all point forward (a DAG, every node of the
  Notations' E class), where DI-CYC ends in finitely many cycles with no
  fluid left (the finite convergence the paper notes for Dataset 2).

Each solve is compared with the CPU oracle's solution within the error
bound of the stopping rule (residual / (1 - d)), as in the main parity
tests.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen

pytestmark = pytest.mark.gpu

D = 0.85
TOL_PAR = 1.4e-10
KERNELS = [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


_BASE = {}


def base(n):
    if n not in _BASE:
        _BASE[n] = graphgen.web_graph(n, seed=0)
    return _BASE[n]


def gpu_x(torch, n, src, dst, kernel=di.DI_KERNEL_PULL, tol=TOL_PAR):
    g = di.Graph(n, src, dst)
    o = di.di_opts_default()
    o.kernel = kernel
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, tol, o, X)
    assert status == di.DI_OK, di.di_last_error()
    torch.cuda.synchronize()
    g.close()
    return X.cpu().numpy(), st


def oracle_x(n, src, dst):
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    H, _, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert st.status == oracle.OK
    return og, B, H


@pytest.mark.parametrize("kernel", KERNELS)
def test_transposed_10k(torch_cuda, kernel):
    n = 10000
    src, dst = graphgen.transpose(*base(n))
    og, B, ref = oracle_x(n, src, dst)
    X, st = gpu_x(torch_cuda, n, src, dst, kernel)
    assert np.abs(X - ref).sum() <= 1e-9
    _, r = oracle.residual(og, B, D, X)
    assert abs(r - st.resid_l1) <= 1e-14


def test_transposed_1m(torch_cuda):
    n = 1_000_000
    src, dst = graphgen.transpose(*base(n))
    stats = graphgen.graph_stats(n, src, dst)
    assert stats.max_out > 50_000  # the hub now sends along all its links
    og, B, ref = oracle_x(n, src, dst)
    X, st = gpu_x(torch_cuda, n, src, dst)
    assert np.abs(X - ref).sum() <= 1e-9
    _, r = oracle.residual(og, B, D, X)
    assert abs(r - st.resid_l1) <= 1e-14


@pytest.mark.parametrize("m", [1000, 3000, 10_000, 30_000, 100_000])
def test_prefix_subgraphs(torch_cuda, m):
    src, dst = graphgen.prefix_subgraph(m, *base(1_000_000))
    og, B, ref = oracle_x(m, src, dst)
    X, st = gpu_x(torch_cuda, m, src, dst)
    assert np.abs(X - ref).sum() <= 1e-9
    _, _, so = oracle.diter(og, B, D, oracle.SOP, oracle.SYNC, tol=TOL_PAR)
    assert abs(st.cycles - so.cycles) <= 1


def test_dag_converges_in_finitely_many_cycles(torch_cuda):
    n = 3000
    src, dst = graphgen.web_graph(n, seed=2, alpha=graphgen.ALPHA_LITERAL, p_dangling=0.48,
                                  p_local=1.0, p_forward=1.0)
    assert np.all(dst > src)
    # longest path in links: an upper bound on the cycles DI-CYC needs
    depth = np.zeros(n, np.int64)
    for a, b in zip(src.tolist(), dst.tolist()):  # sorted by origin: a DAG in id order
        depth[b] = max(depth[b], depth[a] + 1)
    og, B, ref = oracle_x(n, src, dst)
    # one ascending sweep of the oracle's DI-CYC is exact on a forward DAG
    exact, _, ost = oracle.diter(og, B, D, oracle.CYC, oracle.SEQUENTIAL, tol=1e-300)
    assert ost.status == oracle.OK and ost.resid_l1 == 0.0
    g = di.Graph(n, src, dst)
    o = di.di_opts_default()
    o.method = di.DI_CYC
    X = torch_cuda.empty(n, dtype=torch_cuda.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, 1e-300, o, X)
    assert status == di.DI_OK, di.di_last_error()
    torch_cuda.cuda.synchronize()
    assert st.resid_l1 == 0.0 and st.cycles <= int(depth.max()) + 1
    assert np.abs(X.cpu().numpy() - exact).sum() <= 1e-14
    # DI-SOP reaches the tolerance on the same graph as well
    Xs, sts = gpu_x(torch_cuda, n, src, dst)
    assert np.abs(Xs - ref).sum() <= 1e-9
