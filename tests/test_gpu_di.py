"""GPU parity of the FP64 / FP32 DI-SOP path against the CPU oracle.

Every call goes through the C ABI (libdi.so). Expected values come from the
oracle (or closed forms); nothing here is produced by the GPU path itself.
Parity reading: stopping at sum|F| <= tol bounds |X - H|_1 by tol/(1-d);
the parity runs stop at 1.4e-10 so that the bound, plus the oracle's own
1e-13, stays below 1e-9.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen
from tests._sched import schedule_of
from tests._dense import dense_solve

pytestmark = pytest.mark.gpu

D = 0.85
TOL_PAR = 1.4e-10   # (1 - d) * 1e-9 - 1e-13, rounded down
TOL_REF = 1e-13


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def gpu_solve(torch, g, B, d=D, tol=TOL_PAR, allow=(di.DI_OK,), **fields):
    o = di.di_opts_default()
    for k, v in fields.items():
        setattr(o, k, v)
    X = torch.empty(g.n, dtype=torch.float64, device="cuda")
    Bd = None if B is None else torch.from_numpy(np.ascontiguousarray(B, np.float64)).cuda()
    status, st = di.di_solve_dev(g.handle, Bd, d, tol, o, X)
    assert status in allow, (di.STATUS_NAMES.get(status), di.di_last_error())
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, status


def oracle_ref(n, src, dst, B, tol=TOL_REF):
    og = oracle.Graph(n, src, dst)
    H, F, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=tol)
    assert st.status == oracle.OK
    return og, H


_GRAPHS = {}


def web(n, alpha=graphgen.ALPHA_L_MATCHED, kmax=500, seed=0):
    key = (n, alpha, kmax, seed)
    if key not in _GRAPHS:
        _GRAPHS[key] = graphgen.web_graph(n, seed=seed, alpha=alpha, kmax=kmax)
    return _GRAPHS[key]


# ---------------------------------------------------------------- per cycle

def test_worked_example_cycles_sync(torch_cuda):
    """The hand-worked frontier-synchronous cycles of the 4-node example."""
    from tests.test_oracle_pins import _read_worked_example
    from fractions import Fraction
    torch = torch_cuda
    spec, runs = _read_worked_example()
    n = int(spec["n"][0])
    d = float(Fraction(spec["d"][0]))
    links = [tuple(int(x) for x in s.split(":")) for s in spec["links"]]
    src = np.array([a for a, _ in links], np.int32)
    dst = np.array([b for _, b in links], np.int32)
    B = np.array([float(Fraction(v)) for v in spec["B"]])
    g = di.Graph(n, src, dst)
    F = torch.from_numpy(B.copy()).cuda()
    H = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = 0.0
    for c in runs["sync"]:
        H_before = H.cpu().numpy()
        status, e, st = di.di_cycles_dev(g.handle, d, di.DI_SOP, F, H, 1, e)
        assert status == di.DI_OK, di.di_last_error()
        torch.cuda.synchronize()
        Fh, Hh = F.cpu().numpy(), H.cpu().numpy()
        assert list(np.nonzero(Hh != H_before)[0]) == c["selected"]
        assert np.allclose(Fh, c["F"], rtol=0, atol=1e-16), (Fh, c["F"])
        assert np.allclose(Hh, c["H"], rtol=0, atol=1e-16), (Hh, c["H"])
        assert abs(e - c["e"][0]) < 1e-16
        assert st.edges_pushed == c["link_ops"]


@pytest.mark.parametrize("case", ["web10k", "web10k_literal", "loops"])
def test_cycles_match_oracle_sync_schedule(torch_cuda, case):
    """Each GPU cycle selects the same nodes as the oracle's labelled
    frontier-synchronous cycle and leaves the same F and H (to the rounding
    of unordered atomic additions)."""
    torch = torch_cuda
    rng = np.random.default_rng(3)
    if case == "loops":
        n = 3000
        src, dst = web(n, seed=5)
        # add self-loops to every 7th node, keeping (src, dst) order
        extra = np.arange(0, n, 7, dtype=np.int32)
        src = np.concatenate([src, extra])
        dst = np.concatenate([dst, extra])
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
        B = rng.random(n) * 1e-4
    else:
        n = 10000
        src, dst = web(n, alpha=graphgen.ALPHA_LITERAL if case.endswith("literal") else graphgen.ALPHA_L_MATCHED)
        B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    og = oracle.Graph(n, src, dst)
    Fo, Ho, eo = B.copy(), np.zeros(n), 0.0
    F = torch.from_numpy(B.copy()).cuda()
    H = torch.zeros(n, dtype=torch.float64, device="cuda")
    e = 0.0
    scale = B.sum()
    for cyc in range(15):
        H_before = H.cpu().numpy()
        status, e, st = di.di_cycles_dev(g.handle, D, di.DI_SOP, F, H, 1, e)
        assert status == di.DI_OK
        cnt, sel, eo, ops, r = oracle.di_cycle(og, Fo, Ho, D, oracle.SOP, oracle.SYNC, eo)
        torch.cuda.synchronize()
        Fh, Hh = F.cpu().numpy(), H.cpu().numpy()
        gsel = Hh != H_before
        assert np.array_equal(gsel, sel), (cyc, np.nonzero(gsel != sel)[0][:10])
        assert st.edges_pushed == ops
        assert np.abs(Fh - Fo).sum() <= 1e-13 * scale, cyc
        assert np.abs(Hh - Ho).sum() <= 1e-13 * scale, cyc
        assert abs(e - eo) <= 1e-13 * scale


# ------------------------------------------------------------- full solves

KERNELS = [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("seed", range(6))
def test_small_random_graphs_vs_dense(torch_cuda, seed, kernel):
    from tests.test_oracle_pins import _random_graph
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 51))
    src, dst = _random_graph(rng, n)
    if src.size == 0:
        src, dst = np.array([0], np.int32), np.array([1], np.int32)
    B = rng.random(n)
    X_ref, _ = dense_solve(n, src, dst, D, B)
    g = di.Graph(n, src, dst)
    X, st, _ = gpu_solve(torch_cuda, g, B, tol=1e-13, kernel=kernel)
    assert np.abs(X - X_ref).sum() <= 1e-13 / (1 - D) + 1e-13 * X_ref.sum()
    assert st.resid_l1 <= 1e-13


@pytest.mark.parametrize("kernel", KERNELS)
def test_closed_forms(torch_cuda, kernel):
    import functools
    torch = torch_cuda
    gpu_solve_k = functools.partial(gpu_solve, kernel=kernel)
    # directed cycle: X = 1/N
    n = 1000
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    order = np.lexsort((dst, src))
    X, _, _ = gpu_solve_k(torch, di.Graph(n, src[order], dst[order]), None, tol=1e-14)
    assert np.allclose(X, 1.0 / n, rtol=0, atol=1e-15)
    # complete digraph with self-loops: X = 1/N (transit formula)
    n = 40
    src, dst = np.divmod(np.arange(n * n), n)
    X, _, _ = gpu_solve_k(torch, di.Graph(n, src.astype(np.int32), dst.astype(np.int32)), None, tol=1e-15)
    assert np.allclose(X, 1.0 / n, rtol=0, atol=1e-15)
    # chain 0 -> 1: the tie case of the selection rule
    X, st, _ = gpu_solve_k(torch, di.Graph(2, np.array([0], np.int32), np.array([1], np.int32)), None, tol=1e-16)
    assert np.allclose(X, [(1 - D) / 2, (1 - D) * (1 + D) / 2], rtol=0, atol=1e-16)
    assert st.fallback_cycles == 0
    # lone self-loop plus an isolated node
    X, _, _ = gpu_solve_k(torch, di.Graph(2, np.array([0], np.int32), np.array([0], np.int32)),
                        np.array([0.2, 0.3]), tol=1e-16)
    assert abs(X[0] - 0.2 / (1 - D)) < 1e-15 and X[1] == 0.3
    # no links at all: X = B after one cycle
    B = np.linspace(0.1, 1.0, 5)
    X, st, _ = gpu_solve_k(torch, di.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32)), B, tol=1e-16)
    assert np.array_equal(X, B) and st.cycles == 1 and st.edges_pushed == 0
    # single node, no links
    X, _, _ = gpu_solve_k(torch, di.Graph(1, np.zeros(0, np.int32), np.zeros(0, np.int32)), None)
    assert X[0] == 1 - D


@pytest.mark.parametrize("kernel", KERNELS)
def test_star_spans_many_push_tiles(torch_cuda, kernel):
    """One node with 30000 out-links (a frontier entry far longer than a push
    block) and a hub with 30000 in-links (split into 15 pull segments; on
    the push side, all atomics on one address)."""
    n = 30001
    src = np.concatenate([np.zeros(n - 1, np.int64), np.arange(1, n)]).astype(np.int32)
    dst = np.concatenate([np.arange(1, n), np.zeros(n - 1, np.int64)]).astype(np.int32)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    rng = np.random.default_rng(1)
    B = rng.random(n) / n
    og, X_ref = oracle_ref(n, src, dst, B)
    X, st, _ = gpu_solve(torch_cuda, di.Graph(n, src, dst), B, kernel=kernel)
    assert np.abs(X - X_ref).sum() <= 1e-9


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("alpha", [graphgen.ALPHA_L_MATCHED, graphgen.ALPHA_LITERAL])
def test_parity_10k_pagerank(torch_cuda, alpha, kernel):
    n = 10000
    src, dst = web(n, alpha=alpha)
    B = graphgen.uniform_rhs(n, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    g = di.Graph(n, src, dst)
    X, st, _ = gpu_solve(torch_cuda, g, None, kernel=kernel)
    assert np.abs(X - X_ref).sum() <= 1e-9
    # sum |F| is the residual of H: recompute it from X with the oracle
    _, r_true = oracle.residual(og, B, D, X)
    assert abs(r_true - st.resid_l1) <= 1e-14
    # the GPU's schedule does the work of the oracle's matching mode
    sch, kw = schedule_of(g, kernel)
    _, _, so = oracle.diter(og, B, D, oracle.SOP, sch, tol=TOL_PAR, **kw)
    assert abs(st.cycles - so.cycles) <= 1
    assert abs(st.nb_iter - so.nb_iter) <= 0.02 * so.nb_iter


def test_parity_1m_bench_configuration(torch_cuda):
    """N = 1M web graph, uniform B, default options (the benchmark's launch
    configuration), every entry of X compared."""
    n = 1_000_000
    src, dst = web(n)
    B = graphgen.uniform_rhs(n, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    g = di.Graph(n, src, dst)
    X, st, _ = gpu_solve(torch_cuda, g, None)
    assert np.abs(X - X_ref).sum() <= 1e-9
    _, r_true = oracle.residual(og, B, D, X)
    assert abs(r_true - st.resid_l1) <= 1e-14
    # at the headline tolerance the error bound is reported, not gated
    X9, st9, _ = gpu_solve(torch_cuda, g, None, tol=1e-9)
    assert st9.resid_l1 <= 1e-9
    assert np.abs(X9 - X_ref).sum() <= st9.err_bound + 1e-12
    # the default is the tuned window push
    tun = di.di_graph_tuning(g.handle)
    assert tun["tuned"] and tun["tile"] in (1024, 2048, 4096) and 0 <= tun["hubs"] <= 1024
    assert 0 < tun["us_tuned"] <= tun["us_default"] and tun["us_pull"] > 0
    assert tun["kernel"] == ("pull" if tun["us_pull"] < tun["us_tuned"] else "window")
    # the pull direction is bit-reproducible
    Xq, stq, _ = gpu_solve(torch_cuda, g, None, kernel=di.DI_KERNEL_PULL)
    X2, _, _ = gpu_solve(torch_cuda, g, None, kernel=di.DI_KERNEL_PULL)
    assert np.array_equal(X2, Xq)
    assert np.abs(Xq - X_ref).sum() <= 1e-9
    # the default's cycles are those of the oracle's matching schedule (two
    # rounds a cycle over the window's tiles take fewer than the pull's)
    sch, kw = schedule_of(g, di.DI_KERNEL_AUTO)
    _, _, so = oracle.diter(og, B, D, oracle.SOP, sch, tol=TOL_PAR, **kw)
    assert abs(st.cycles - so.cycles) <= 1
    # the push differs from the pull only by the order of atomic additions
    Xp, stp, _ = gpu_solve(torch_cuda, g, None, kernel=di.DI_KERNEL_PUSH)
    assert np.abs(Xp - X_ref).sum() <= 1e-9
    assert np.abs(Xp - Xq).sum() <= 1e-12
    assert stp.cycles == stq.cycles


@pytest.mark.parametrize("kernel", KERNELS)
def test_fp32_fluid(torch_cuda, kernel):
    n = 10000
    src, dst = web(n)
    B = graphgen.uniform_rhs(n, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    X, st, _ = gpu_solve(torch_cuda, di.Graph(n, src, dst), None, tol=1e-7, precision=di.DI_FP32,
                         kernel=kernel)
    assert np.abs(X - X_ref).sum() <= 2e-6 * X_ref.sum()


@pytest.mark.parametrize("kernel", [di.DI_KERNEL_PULL, di.DI_KERNEL_WINDOW])
def test_fp32_fluid_at_1m(torch_cuda, kernel):
    """Plain FP32 fluid at the benchmark size: within 2e-6 |X|_1 of the
    oracle's FP64 solution."""
    n = 1_000_000
    src, dst = web(n)
    B = graphgen.uniform_rhs(n, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    X, st, _ = gpu_solve(torch_cuda, di.Graph(n, src, dst), None, tol=1e-7, precision=di.DI_FP32,
                         kernel=kernel)
    assert np.abs(X - X_ref).sum() <= 2e-6 * X_ref.sum()


@pytest.mark.parametrize("kernel", KERNELS)
def test_paper_stop_same_cycle_as_oracle_sync(torch_cuda, kernel):
    """The paper's stop rule (sum F / (1 - d - d e) <= 1/N, Section 2.5.4):
    the GPU stops on the same cycle as the oracle's run in the matching
    schedule (frontier-synchronous, or tiled for the window push) and
    reports the same estimate to rounding."""
    n = 10000
    src, dst = web(n)
    B = graphgen.uniform_rhs(n, D)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    X, st, _ = gpu_solve(torch_cuda, g, None, tol=1.0 / n, stop=di.DI_STOP_PAPER, kernel=kernel)
    sch, kw = schedule_of(g, kernel)
    _, _, so = oracle.diter(og, B, D, oracle.SOP, sch, stop=oracle.STOP_PAPER, tol=1.0 / n, **kw)
    assert st.cycles == so.cycles
    assert abs(st.paper_err - so.paper_err) <= 1e-12 * so.paper_err
    assert abs(st.e - so.e) <= 1e-12 * so.e


def test_cyc_method_and_paper_stop(torch_cuda):
    n = 10000
    src, dst = web(n)
    B = graphgen.uniform_rhs(n, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    g = di.Graph(n, src, dst)
    X, st, _ = gpu_solve(torch_cuda, g, None, method=di.DI_CYC)
    assert np.abs(X - X_ref).sum() <= 1e-9
    _, _, so = oracle.diter(og, B, D, oracle.CYC, oracle.SYNC, tol=TOL_PAR)
    assert abs(st.cycles - so.cycles) <= 1
    # the paper's stopping rule with target 1/N
    X, st, _ = gpu_solve(torch_cuda, g, None, tol=1.0 / n, stop=di.DI_STOP_PAPER)
    assert st.paper_err <= 1.0 / n
    xn = X_ref / X_ref.sum()
    assert np.abs(X / X.sum() - xn).sum() <= 2.0 / n


def test_host_entry_point_and_personalized_b(torch_cuda):
    n = 10000
    src, dst = web(n)
    g = di.Graph(n, src, dst)
    seeds = graphgen.ppr_seed_sets(n, 1)[0]
    B = graphgen.ppr_rhs(n, seeds, D)
    og, X_ref = oracle_ref(n, src, dst, B)
    X, st = di.solve(g, B, D, TOL_PAR)
    assert np.abs(X - X_ref).sum() <= 1e-9
    Xd, _, _ = gpu_solve(torch_cuda, g, B)
    assert np.abs(X - Xd).sum() <= 1e-12


def test_signed_right_hand_side(torch_cuda):
    rng = np.random.default_rng(12)
    n = 5000
    src, dst = web(n, seed=9)
    B = rng.standard_normal(n) * 1e-4
    og, X_ref = oracle_ref(n, src, dst, B)
    X, _, _ = gpu_solve(torch_cuda, di.Graph(n, src, dst), B)
    assert np.abs(X - X_ref).sum() <= 1e-9


@pytest.mark.parametrize("kernel", KERNELS)
def test_max_cycles_stops_on_an_exact_prefix(torch_cuda, kernel):
    """A solve stopped by max_cycles returns the history of exactly that many
    cycles, at and around the host's read-back points (the first after 8
    cycles), although the host keeps a cycle queued behind each read-back:
    the pull's bit for bit that of di_cycles_dev, the others' that of the
    oracle's matching schedule to rounding."""
    torch = torch_cuda
    n = 10000
    src, dst = web(n)
    g = di.Graph(n, src, dst)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    for m in (1, 2, 8, 9, 10, 23):
        X, st, status = gpu_solve(torch, g, None, tol=1e-15, allow=(di.DI_E_NOCONV,), max_cycles=m,
                                  kernel=kernel)
        assert status == di.DI_E_NOCONV and st.cycles == m, (m, st.cycles)
        sch, kw = schedule_of(g, kernel)
        if sch != oracle.SYNC:
            Ho, _, so = oracle.diter(og, B, D, oracle.SOP, sch, tol=0.0, max_cycles=m, **kw)
            assert so.cycles == m and np.abs(X - Ho).sum() <= 1e-13, m
            continue
        F = torch.from_numpy(B.copy()).cuda()
        H = torch.zeros(n, dtype=torch.float64, device="cuda")
        status, _, stc = di.di_cycles_dev(g.handle, D, di.DI_SOP, F, H, m)
        assert status == di.DI_OK and stc.cycles == m
        torch.cuda.synchronize()
        Hh = H.cpu().numpy()
        if kernel == di.DI_KERNEL_PULL:
            assert np.array_equal(X, Hh), m
        else:  # atomic order differs between runs
            assert np.abs(X - Hh).sum() <= 1e-13, m


def test_errors_on_device(torch_cuda):
    torch = torch_cuda
    n = 1000
    src, dst = web(n)
    g = di.Graph(n, src, dst)
    # max_cycles reached
    X, st, status = gpu_solve(torch, g, None, tol=1e-15, allow=(di.DI_E_NOCONV,), max_cycles=3)
    assert status == di.DI_E_NOCONV and st.cycles == 3
    # non-finite B: rejected on the host for di_solve, on the device for _dev
    B = np.full(n, 1e-3)
    B[17] = np.nan
    Xh = np.empty(n)
    status, _ = di.di_solve(g.handle, B, D, 1e-9, None, Xh)
    assert status == di.DI_E_INVAL
    _, _, status = gpu_solve(torch, g, B, allow=(di.DI_E_INVAL,))
    assert status == di.DI_E_INVAL
    # bad d / tol
    for dd, tt in ((1.0, 1e-9), (0.0, 1e-9), (0.85, 0.0), (0.85, -1.0)):
        status, _ = di.di_solve(g.handle, None, dd, tt, None, Xh)
        assert status == di.DI_E_INVAL
