"""Per-cycle trace of a solve (di_solve_trace_dev): each record against the
hand-worked cycles of the 4-node example and against the oracle's cycles in
the schedule the GPU runs (Section 2.5.5 selection, one r per cycle):
frontier-synchronous, or tiled with two rounds for DI-SOP on the window
push."""
import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen
from tests._sched import schedule_of
from tests.test_oracle_pins import _read_worked_example

pytestmark = pytest.mark.gpu

D = 0.85
TOL = 1.4e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def traced(torch, g, B, capacity, d=D, tol=TOL, allow=(di.DI_OK,), **fields):
    o = di.di_opts_default()
    for k, v in fields.items():
        setattr(o, k, v)
    X = torch.empty(g.n, dtype=torch.float64, device="cuda")
    Bd = None if B is None else torch.from_numpy(np.ascontiguousarray(B, np.float64)).cuda()
    status, st, recs = di.di_solve_trace_dev(g.handle, Bd, d, tol, o, X, capacity)
    assert status in allow, (di.STATUS_NAMES.get(status), di.di_last_error())
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, recs


def test_trace_worked_example(torch_cuda):
    """The records of the first cycles equal the hand-worked ones: r is the
    sum of F before the cycle, selected and link operations as worked."""
    from fractions import Fraction
    spec, runs = _read_worked_example()
    n = int(spec["n"][0])
    d = float(Fraction(spec["d"][0]))
    links = [tuple(int(x) for x in s.split(":")) for s in spec["links"]]
    src = np.array([a for a, _ in links], np.int32)
    dst = np.array([b for _, b in links], np.int32)
    B = np.array([float(Fraction(v)) for v in spec["B"]])
    g = di.Graph(n, src, dst)
    worked = runs["sync"]
    # a tolerance far below the worked cycles: the capacity cuts the trace
    # (the worked cycles are frontier-synchronous: the pull's schedule)
    _, st, recs = traced(torch_cuda, g, B, len(worked), d=d, tol=1e-14,
                         kernel=di.DI_KERNEL_PULL)
    assert st.cycles > len(worked)
    assert len(recs) == len(worked)
    F_prev = B
    for c, (rec, w) in enumerate(zip(recs, worked)):
        assert abs(rec.r - np.abs(F_prev).sum()) <= 1e-16, c
        assert rec.selected == len(w["selected"]), c
        assert rec.links == w["link_ops"], c
        F_prev = np.array(w["F"])


@pytest.mark.parametrize("kernel", [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW])
@pytest.mark.parametrize("alpha", [graphgen.ALPHA_L_MATCHED, graphgen.ALPHA_LITERAL])
def test_trace_matches_oracle_cycles(torch_cuda, alpha, kernel):
    """Every record of a whole solve on a 10k web graph equals the oracle's
    cycle in the same schedule from the same state: the same diffusions, the
    same link operations, r to rounding."""
    n = 10000
    src, dst = graphgen.web_graph(n, seed=0, alpha=alpha, kmax=500)
    B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, B, 4096, kernel=kernel)
    assert len(recs) == st.cycles > 10
    assert sum(r.links for r in recs) == st.edges_pushed
    og = oracle.Graph(n, src, dst)
    sch, kw = schedule_of(g, kernel)
    # links each node moves when diffused (self-loops stay)
    moves = np.bincount(src[src != dst], minlength=n) > 0
    F, H, e = B.copy(), np.zeros(n), 0.0
    for c, rec in enumerate(recs):
        cnt, sel, e, ops, r = oracle.di_cycle(og, F, H, D, oracle.SOP, sch, e, **kw)
        assert abs(rec.r - r) <= 1e-13 * r, (c, rec.r, r)
        assert rec.selected == cnt, c
        assert rec.links == ops, c
        if sch == oracle.SYNC:  # one diffusion per node and cycle
            assert cnt == int(sel.sum()), c
            assert rec.senders == int(np.count_nonzero(sel & moves)), c
    # the solve stopped at the first cycle whose start is within tol
    assert np.abs(F).sum() <= TOL < recs[-1].r


@pytest.mark.parametrize("kernel", [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW])
def test_trace_dicyc_matches_oracle_cycles(torch_cuda, kernel):
    """DI-CYC: every record equals the oracle's frontier-synchronous DI-CYC
    cycle (every node holding fluid diffused) from the same state."""
    n = 10000
    src, dst = graphgen.web_graph(n, seed=3)
    B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, B, 4096, kernel=kernel, method=di.DI_CYC)
    assert len(recs) == st.cycles > 10
    og = oracle.Graph(n, src, dst)
    moves = np.bincount(src[src != dst], minlength=n) > 0
    F, H, e = B.copy(), np.zeros(n), 0.0
    for c, rec in enumerate(recs):
        held = int(np.count_nonzero(F))
        cnt, sel, e, ops, r = oracle.di_cycle(og, F, H, D, oracle.CYC, oracle.SYNC, e)
        assert abs(rec.r - r) <= 1e-13 * r, (c, rec.r, r)
        assert rec.selected == cnt == held, c
        assert rec.links == ops, c
        assert rec.senders == int(np.count_nonzero(sel & moves)), c
    assert np.abs(F).sum() <= TOL < recs[-1].r


def test_trace_matches_oracle_cycles_at_1m(torch_cuda):
    """The benchmark's configuration (N = 1M web graph, uniform B, default
    options): every cycle of the whole solve diffuses exactly the oracle's
    selections in the same schedule (the tuned window push: two rounds a
    cycle over its tiles), with r to rounding."""
    n = 1_000_000
    src, dst = graphgen.web_graph(n, seed=0)
    B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, None, 4096)
    assert len(recs) == st.cycles > 40
    og = oracle.Graph(n, src, dst)
    sch, kw = schedule_of(g, di.DI_KERNEL_AUTO)
    F, H, e = B.copy(), np.zeros(n), 0.0
    for c, rec in enumerate(recs):
        cnt, sel, e, ops, r = oracle.di_cycle(og, F, H, D, oracle.SOP, sch, e, **kw)
        # the oracle adds N terms one after another: within (N - 1) u of the sum
        assert abs(rec.r - r) <= (n - 1) * 0.5 * np.finfo(float).eps * r, (c, rec.r, r)
        assert rec.selected == cnt and rec.links == ops, c
    assert np.abs(F).sum() <= TOL < recs[-1].r


def test_trace_capacity_prefix(torch_cuda):
    """A short trace is the prefix of the full one (the pull is
    bit-reproducible); capacity 0 writes nothing and still solves."""
    n = 10000
    src, dst = graphgen.web_graph(n, seed=1)
    g = di.Graph(n, src, dst)
    pull = di.DI_KERNEL_PULL
    X_full, st, full = traced(torch_cuda, g, None, 4096, kernel=pull)
    X_part, _, part = traced(torch_cuda, g, None, 7, kernel=pull)
    X_none, st0, none = traced(torch_cuda, g, None, 0, kernel=pull)
    assert len(part) == 7 and none == []
    for a, b in zip(part, full):
        assert (a.r, a.links, a.selected, a.senders) == (b.r, b.links, b.selected, b.senders)
    assert np.array_equal(X_part, X_full) and np.array_equal(X_none, X_full)
    assert st0.cycles == st.cycles


def test_trace_fp32_refine_numbers_passes_in_order(torch_cuda):
    """FP32 with FP64 refinement: the passes' cycles follow one another in
    the trace, and every record's r is that of an FP32 pass (each pass
    starts from the residual recomputed in FP64, so r jumps up at most to
    the previous pass's stop)."""
    n = 10000
    src, dst = graphgen.web_graph(n, seed=2)
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, None, 4096, tol=1e-9, precision=di.DI_FP32_REFINE)
    assert st.refinements >= 1
    assert len(recs) == st.cycles
    assert sum(r.links for r in recs) == st.edges_pushed
    r = np.array([x.r for x in recs])
    assert r[0] == pytest.approx(1.0 - D, rel=1e-6)
    # within a pass r falls (F >= 0 loses a share of each diffusion); it can
    # rise only where a pass starts from the FP64 residual
    rises = np.nonzero(r[1:] > r[:-1])[0] + 1
    assert len(rises) <= st.refinements
    # no cycle started below the inner stop (0.9 of the tolerance)
    assert r.min() > 0.9e-9


def test_trace_pi_diffuses_every_node(torch_cuda):
    """DI_PI: every cycle diffuses all n nodes and moves every link."""
    n = 5000
    src, dst = graphgen.web_graph(n, seed=4)
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, None, 4096, tol=1e-8, method=di.DI_PI)
    assert len(recs) == st.cycles
    moved = int(np.count_nonzero(src != dst))
    for rec in recs:
        assert rec.selected == n
        assert rec.links == moved
    r = np.array([x.r for x in recs])
    assert np.all(r[1:] < r[:-1])


@pytest.mark.parametrize("kernel", [di.DI_KERNEL_PULL, di.DI_KERNEL_PUSH, di.DI_KERNEL_WINDOW])
def test_trace_pi_r_is_the_norm_of_matrix_powers(torch_cuda, kernel):
    """DI_PI diffuses every node each cycle, so the fluid at the start of cycle
    c is P^c.B: each record's r equals |P^c B|_1, computed with the oracle's
    product by P."""
    n = 5000
    src, dst = graphgen.web_graph(n, seed=6)
    rng = np.random.default_rng(6)
    B = rng.random(n) * (1.0 - D) / n
    g = di.Graph(n, src, dst)
    _, st, recs = traced(torch_cuda, g, B, 4096, tol=1e-10, method=di.DI_PI, kernel=kernel)
    assert len(recs) == st.cycles > 20
    og = oracle.Graph(n, src, dst)
    x = B.copy()
    for c, rec in enumerate(recs):
        want = np.abs(x).sum()
        # sums of up to a hub's in-degree of terms, in another order, per cycle
        assert abs(rec.r - want) <= (c + 1) * 1e-13 * want, (c, rec.r, want)
        x = oracle.apply_p(og, D, x)


def test_trace_rejects(torch_cuda):
    torch = torch_cuda
    n = 100
    src, dst = graphgen.web_graph(n, seed=5)
    g = di.Graph(n, src, dst)
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    o = di.di_opts_default()
    o.method = di.DI_GS_ASYNC
    status, _, recs = di.di_solve_trace_dev(g.handle, None, D, 1e-9, o, X, 16)
    assert status == di.DI_E_INVAL and recs == []
    status, _, _ = di.di_solve_trace_dev(g.handle, None, D, 1e-9, None, X, -1)
    assert status == di.DI_E_INVAL
