"""GPU parity on two more workloads of the paper's kind:

- the transposed web graph (Section 2.7, Dataset 1bis: the same graph
  with every link reversed), where the generator's in-degree hubs become
  nodes with tens of thousands of out-links;
- prefix subgraphs of the N = 1M graph (the subgraph induced on the node
  ids below m), the paper's way of varying N (Section 2.6, Table 1).

- a graph whose links all point forward (a DAG, every node of the
  Notations' E class), where DI-CYC ends in finitely many cycles with no
  fluid left (the finite convergence the paper notes for Dataset 2);
- the stand-in for Dataset 2 (Section 2.8, Table 9: 91% of the nodes in the
  E class) and its transpose, where every E node of depth h holds no fluid
  after h + 1 synchronous DI-CYC cycles;
- DI-CYC run for m + 1 cycles against the oracle's power iteration after m
  steps: with every node holding fluid diffused each cycle, the GPU's
  history is the PI iterate (pull: rows gathered, as PI of Section 2.5.1;
  push: columns scattered, as PI' of Section 2.5.2), started from zero.

Each solve is compared with the CPU oracle's solution within the error
bound of the stopping rule (residual / (1 - d)), as in the main parity
tests.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen
from _peel import e_depth

pytestmark = pytest.mark.gpu

D = 0.85
TOL_PAR = 1.4e-10
KERNELS = [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW]


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


N_CAL = 9664  # Table 9


@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("method", [di.DI_SOP, di.DI_CYC])
@pytest.mark.parametrize("kernel", KERNELS)
def test_high_e_graph(torch_cuda, transposed, method, kernel):
    src, dst = graphgen.high_e_graph(N_CAL, seed=0)
    if transposed:
        src, dst = graphgen.transpose(src, dst)
    og, B, ref = oracle_x(N_CAL, src, dst)
    g = di.Graph(N_CAL, src, dst)
    o = di.di_opts_default()
    o.kernel = kernel
    o.method = method
    X = torch_cuda.empty(N_CAL, dtype=torch_cuda.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, TOL_PAR, o, X)
    assert status == di.DI_OK, di.di_last_error()
    torch_cuda.cuda.synchronize()
    X = X.cpu().numpy()
    g.close()
    assert np.abs(X - ref).sum() <= 1e-9
    _, r = oracle.residual(og, B, D, X)
    assert abs(r - st.resid_l1) <= 1e-14


@pytest.mark.parametrize("transposed", [False, True])
def test_high_e_nodes_finish_after_their_depth(torch_cuda, transposed):
    torch = torch_cuda
    src, dst = graphgen.high_e_graph(N_CAL, seed=0)
    if transposed:
        src, dst = graphgen.transpose(src, dst)
    depth = e_depth(N_CAL, src, dst)
    assert (depth >= 0).sum() > N_CAL // 2
    og = oracle.Graph(N_CAL, src, dst)
    B = graphgen.uniform_rhs(N_CAL, D)
    Fo, Ho = B.copy(), np.zeros(N_CAL)
    g = di.Graph(N_CAL, src, dst)
    Fd = torch.from_numpy(B.copy()).cuda()
    Hd = torch.zeros(N_CAL, dtype=torch.float64, device="cuda")
    e_o = e_g = 0.0
    for c in range(1, int(depth.max()) + 3):
        _, _, e_o, _, _ = oracle.di_cycle(og, Fo, Ho, D, oracle.CYC, oracle.SYNC, e_o)
        status, e_g, _ = di.di_cycles_dev(g.handle, D, di.DI_CYC, Fd, Hd, 1, e_g)
        assert status == di.DI_OK, di.di_last_error()
        torch.cuda.synchronize()
        F, H = Fd.cpu().numpy(), Hd.cpu().numpy()
        done = (depth >= 0) & (depth < c)
        assert np.all(F[done] == 0.0), (c, np.abs(F[done]).max())
        # same schedule as the oracle's SYNC mode, sums in another order
        assert np.all(np.abs(F - Fo) <= 1e-16 + 1e-13 * np.abs(Fo)), c
        assert np.all(np.abs(H - Ho) <= 1e-16 + 1e-13 * np.abs(Ho)), c
        assert abs(e_g - e_o) <= 1e-13 * max(abs(e_o), 1e-300), c
    g.close()


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("m", [0, 3, 17])
def test_cyc_is_the_power_iteration(torch_cuda, kernel, m):
    n = 10000
    src, dst = base(n)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    x_pi, st_pi = oracle.jacobi(og, B, D, tol=0.0, max_iter=m)
    assert st_pi.status == oracle.E_NOCONV and st_pi.cycles == m
    g = di.Graph(n, src, dst)
    o = di.di_opts_default()
    o.kernel = kernel
    o.method = di.DI_CYC
    o.max_cycles = m + 1
    X = torch_cuda.empty(n, dtype=torch_cuda.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, 1e-300, o, X)
    assert status == di.DI_E_NOCONV and st.cycles == m + 1, di.di_last_error()
    torch_cuda.cuda.synchronize()
    g.close()
    X = X.cpu().numpy()
    # a cycle moves at most every link once (nodes without in-links hold no
    # fluid after the first cycle, while PI still pays for their links)
    assert 0 < st.edges_pushed <= (m + 1) * len(src)
    # all terms are positive: the two summation orders differ by a few ulps
    # per step, relative to the entry
    eps = np.finfo(float).eps
    assert np.all(np.abs(X - x_pi) <= (m + 1) * 4 * (np.log2(n) + 8) * eps * x_pi)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_pi_method_is_the_power_iteration(torch_cuda, kernel, tol):
    """DI_PI diffuses every node every cycle: after c cycles H is the power
    iteration's iterate x_{c-1} (from x_0 = B) and sum|F| = |P^c B|_1 its
    residual, so it stops exactly where the oracle's power iteration stops,
    one cycle later by count, with every link moved every cycle."""
    n = 10000
    src, dst = base(n)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    x_pi, st_pi = oracle.jacobi(og, B, D, tol=tol)
    assert st_pi.status == oracle.OK
    g = di.Graph(n, src, dst)
    o = di.di_opts_default()
    o.kernel = kernel
    o.method = di.DI_PI
    X = torch_cuda.empty(n, dtype=torch_cuda.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, tol, o, X)
    assert status == di.DI_OK, di.di_last_error()
    torch_cuda.cuda.synchronize()
    X = X.cpu().numpy()
    m = st_pi.cycles
    assert st.cycles == m + 1
    assert st.edges_pushed == st.cycles * np.count_nonzero(src != dst)
    eps = np.finfo(float).eps
    assert np.all(np.abs(X - x_pi) <= (m + 1) * 4 * (np.log2(n) + 8) * eps * x_pi)
    # the oracle's residual is a difference of nearly equal iterates (its
    # rounding is relative to x); the GPU's is the fluid itself
    assert abs(st.resid_l1 - st_pi.resid_l1) <= 1e-4 * st_pi.resid_l1
    # the batched path and serving take DI_SOP and DI_CYC only
    status, _, _ = di.di_solve_batch(g.handle, 2, None, D, [tol, tol], o)
    assert status == di.DI_E_INVAL
    st_s, h = di.di_serve_create(1 << 30, 8, o)
    assert st_s == di.DI_E_INVAL
    g.close()


def star_graph(n):
    """Node 0 links to every other node and every other node links to 0:
    a row of n - 1 in-links, split into segments by the pull items."""
    src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)]).astype(np.int32)
    dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)]).astype(np.int32)
    order = np.lexsort((dst, src))
    return src[order], dst[order]


def with_loops(n, src, dst, every=7):
    keep = src != dst
    s = np.concatenate([src[keep], np.arange(0, n, every, dtype=np.int32)])
    t = np.concatenate([dst[keep], np.arange(0, n, every, dtype=np.int32)])
    order = np.lexsort((t, s))
    return s[order].astype(np.int32), t[order].astype(np.int32)


@pytest.mark.parametrize("case", ["web10k", "ppr", "signed", "loops", "star", "transposed"])
def test_gs_async(torch_cuda, case):
    """The Gauss-Seidel baseline as an asynchronous GPU relaxation: its
    reported residual is exact and within tol, X is within tol / (1 - d) of
    the oracle's solution, and it needs no more sweeps than the power
    iteration (plus the sweeps the stop test's bound costs)."""
    n = 10000
    if case == "star":
        n = 30001
        src, dst = star_graph(n)
    else:
        src, dst = base(n)
        if case == "loops":
            src, dst = with_loops(n, src, dst)
        elif case == "transposed":
            src, dst = graphgen.transpose(src, dst)
    og = oracle.Graph(n, src, dst)
    if case == "ppr":
        B = graphgen.ppr_rhs(n, graphgen.ppr_seed_sets(n, 1)[0], D)
    elif case == "signed":
        B = np.random.default_rng(3).standard_normal(n) * 1e-4
    else:
        B = graphgen.uniform_rhs(n, D)
    ref, _, ost = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert ost.status == oracle.OK
    g = di.Graph(n, src, dst)
    o = di.di_opts_default()
    o.method = di.DI_GS_ASYNC
    Bd = torch_cuda.from_numpy(np.ascontiguousarray(B)).cuda()
    X = torch_cuda.empty(n, dtype=torch_cuda.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, Bd, D, TOL_PAR, o, X)
    assert status == di.DI_OK, di.di_last_error()
    torch_cuda.cuda.synchronize()
    X = X.cpu().numpy()
    _, r = oracle.residual(og, B, D, X)
    # both residuals are sums of cancelling terms; the oracle adds a row's
    # in-links one after another, whose rounding grows with the in-degree
    indeg = np.bincount(dst[src != dst], minlength=n) + 2
    scale = np.abs(B) + np.abs(X) + oracle.apply_p(og, D, np.abs(X))
    bound = np.finfo(float).eps * float((indeg * scale).sum())
    assert st.resid_l1 <= TOL_PAR and abs(r - st.resid_l1) <= 1e-6 * r + bound
    assert np.abs(X - ref).sum() <= TOL_PAR / (1 - D) + 1e-12
    _, sj = oracle.jacobi(og, B, D, tol=TOL_PAR)
    assert 1 <= st.cycles <= sj.cycles + 3
    assert st.edges_pushed == st.cycles * np.count_nonzero(src != dst)
    # FP64 pull only; not a D-iteration, so no batches, serving or cycles
    o.precision = di.DI_FP32_REFINE
    status, _ = di.di_solve_dev(g.handle, Bd, D, TOL_PAR, o, X := torch_cuda.empty(
        n, dtype=torch_cuda.float64, device="cuda"))
    assert status == di.DI_E_INVAL
    F = torch_cuda.from_numpy(np.ascontiguousarray(B)).cuda()
    H = torch_cuda.zeros(n, dtype=torch_cuda.float64, device="cuda")
    status, _, _ = di.di_cycles_dev(g.handle, D, di.DI_GS_ASYNC, F, H, 1)
    assert status == di.DI_E_INVAL
    g.close()


def test_pi_and_gs_edge_cases(torch_cuda):
    torch = torch_cuda
    n = 10000
    src, dst = base(n)
    og, B, ref = oracle_x(n, src, dst)
    g = di.Graph(n, src, dst)
    # PI with FP32 fluid and FP64 residual passes
    o = di.di_opts_default()
    o.method = di.DI_PI
    o.precision = di.DI_FP32_REFINE
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    status, st = di.di_solve_dev(g.handle, None, D, TOL_PAR, o, X)
    assert status == di.DI_OK and st.refinements >= 1, di.di_last_error()
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    _, r = oracle.residual(og, B, D, Xh)
    assert st.resid_l1 <= TOL_PAR and abs(r - st.resid_l1) <= 1e-15 + 1e-6 * r
    assert np.abs(Xh - ref).sum() <= TOL_PAR / (1 - D) + 1e-12
    # GS-async: max_cycles gives NOCONV with the sweeps' x and its residual
    o = di.di_opts_default()
    o.method = di.DI_GS_ASYNC
    o.max_cycles = 3
    status, st = di.di_solve_dev(g.handle, None, D, 1e-12, o, X)
    assert status == di.DI_E_NOCONV and st.cycles == 3
    torch.cuda.synchronize()
    _, r = oracle.residual(og, B, D, X.cpu().numpy())
    assert abs(r - st.resid_l1) <= 1e-15 + 1e-6 * r and r > 1e-12
    # host arrays, personalized B
    o.max_cycles = 0
    Bp = graphgen.ppr_rhs(n, graphgen.ppr_seed_sets(n, 1, 77)[0], D)
    Xp = np.empty(n)
    status, st = di.di_solve(g.handle, Bp, D, TOL_PAR, o, Xp)
    assert status == di.DI_OK
    refp, _, _ = oracle.diter(og, Bp, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert np.abs(Xp - refp).sum() <= TOL_PAR / (1 - D) + 1e-12
    # B = 0: x = 0 after one sweep, residual 0
    status, st = di.di_solve(g.handle, np.zeros(n), D, TOL_PAR, o, Xp)
    assert status == di.DI_OK and st.cycles == 1 and st.resid_l1 == 0.0 and not Xp.any()
    g.close()
    # one node without links: x = B
    g1 = di.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    X1 = np.empty(1)
    status, st = di.di_solve(g1.handle, None, D, 1e-12, o, X1)
    assert status == di.DI_OK and abs(X1[0] - (1 - D)) <= 1e-16 and st.resid_l1 == 0.0
    # a self-loop-only node: x = B / (1 - d)
    g2 = di.Graph(1, np.zeros(1, np.int32), np.zeros(1, np.int32))
    status, st = di.di_solve(g2.handle, None, D, 1e-12, o, X1)
    assert status == di.DI_OK and abs(X1[0] - 1.0) <= 1e-15
    g1.close()
    g2.close()
