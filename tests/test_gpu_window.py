"""GPU parity of the window push (DI_KERNEL_WINDOW) against the CPU oracle,
through the C ABI.

The window push keeps a cycle's fluid in four places (what a node kept plus
its own tile's near pushes in F, the far accumulator, the neighbours' halos
and the hub partials), so these tests aim at the seams: links at distances
W - 1, W and W + 1 across tile boundaries, graphs of one tile plus or minus
one node, hub rows, self-loops at tile edges, signed and refined fluids, and
the benchmark configuration. Every record of a traced solve is compared with
the oracle's cycle in the schedule the window push runs, from the same
state (Section 2.5.5: the same diffusions and links moved, r to rounding):
for DI-SOP two rounds a cycle over each tile (the oracle's TILED schedule,
with the graph's tile), for DI-CYC and PI the frontier-synchronous cycle.
"""

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen
from tests._sched import schedule_of

pytestmark = pytest.mark.gpu

D = 0.85
TOL_PAR = 1.4e-10
WINDOW = di.DI_KERNEL_WINDOW
TILE = 2048     # nodes per window tile
HALO = 512      # near links: |i - j| <= HALO


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def seam_graph(n, seed):
    """Links at the window's seams: offsets 1, HALO - 1, HALO, HALO + 1 both
    ways, random far links, a hub that many nodes link to from afar,
    dangling nodes and self-loops on every 11th node."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    offs = np.array([1, -1, HALO - 1, -(HALO - 1), HALO, -HALO, HALO + 1, -(HALO + 1)])
    hub = n // 3
    for i in range(n):
        if rng.random() < 0.12:
            continue  # dangling
        k = int(rng.integers(1, 9))
        js = list(i + rng.choice(offs, size=min(k, len(offs)), replace=False))
        js += list(rng.integers(0, n, size=int(rng.integers(0, 4))))
        if abs(i - hub) > HALO and rng.random() < 0.5:
            js.append(hub)
        if i % 11 == 0:
            js.append(i)
        for j in js:
            if 0 <= j < n:
                src.append(i)
                dst.append(int(j))
    key = np.unique(np.array(src, np.int64) * n + np.array(dst, np.int64))
    return (key // n).astype(np.int32), (key % n).astype(np.int32)


def traced(torch, g, B, capacity, tol=TOL_PAR, **fields):
    o = di.di_opts_default()
    o.kernel = WINDOW
    for k, v in fields.items():
        setattr(o, k, v)
    X = torch.empty(g.n, dtype=torch.float64, device="cuda")
    Bd = None if B is None else torch.from_numpy(np.ascontiguousarray(B, np.float64)).cuda()
    status, st, recs = di.di_solve_trace_dev(g.handle, Bd, D, tol, o, X, capacity)
    assert status == di.DI_OK, (di.STATUS_NAMES.get(status), di.di_last_error())
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, recs


def check_against_oracle(og, g, B, recs, variant=oracle.SOP, rtol_r=1e-13):
    method = di.DI_SOP if variant == oracle.SOP else di.DI_CYC
    sch, kw = schedule_of(g, WINDOW, method)
    F, H, e = B.copy(), np.zeros(og.n), 0.0
    for c, rec in enumerate(recs):
        cnt, sel, e, ops, r = oracle.di_cycle(og, F, H, D, variant, sch, e, **kw)
        assert abs(rec.r - r) <= rtol_r * r, (c, rec.r, r)
        assert rec.selected == cnt, (c, rec.selected, cnt)
        assert rec.links == ops, (c, rec.links, ops)
    return H


def pin_rounds(g, rounds):
    """The default window configuration with `rounds` rounds a cycle."""
    t = di.di_graph_tuning(g.handle)
    assert di.di_graph_set_window(g.handle, t["tile"], t["hubs"], 1024, rounds) == di.DI_OK


@pytest.mark.parametrize("rounds", [1, 2])
@pytest.mark.parametrize("n", [TILE - 1, TILE, TILE + 1, 3 * TILE + 5])
def test_seams_every_cycle_and_solution(torch_cuda, n, rounds):
    src, dst = seam_graph(n, seed=n)
    print(f"window seams: n={n} links={src.size} rounds={rounds}", flush=True)
    og = oracle.Graph(n, src, dst)
    rng = np.random.default_rng(n)
    B = rng.random(n) * (1 - D) / n
    g = di.Graph(n, src, dst)
    pin_rounds(g, rounds)
    X, st, recs = traced(torch_cuda, g, B, 4096)
    assert len(recs) == st.cycles > 5
    assert sum(r.links for r in recs) == st.edges_pushed
    check_against_oracle(og, g, B, recs)
    X_ref, _, so = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    assert np.abs(X - X_ref).sum() <= 1e-9
    _, r_true = oracle.residual(og, B, D, X)
    assert st.resid_l1 <= TOL_PAR
    assert abs(r_true - st.resid_l1) <= 1e-14


@pytest.mark.parametrize("method", [di.DI_CYC, di.DI_PI])
def test_seams_cyc_and_pi(torch_cuda, method):
    n = 3 * TILE + 5
    src, dst = seam_graph(n, seed=7)
    if method == di.DI_PI:
        # without self-loops: the transit formula sums a self-loop's series,
        # which the power iteration does one step at a time
        keep = src != dst
        src, dst = src[keep], dst[keep]
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    X, st, recs = traced(torch_cuda, g, B, 4096, tol=1e-11, method=method)
    if method == di.DI_CYC:
        check_against_oracle(og, g, B, recs, variant=oracle.CYC)
        assert np.abs(X - oracle.diter(og, B, D, oracle.SOP, tol=1e-13)[0]).sum() <= 1e-10
    else:
        # every node diffused each cycle: the history after m + 1 cycles is the
        # power iteration's iterate after m steps
        for rec in recs:
            assert rec.selected == n
        x, sj = oracle.jacobi(og, B, D, tol=1e-11)
        assert st.cycles == sj.cycles + 1
        eps = np.finfo(float).eps
        m = sj.cycles
        assert np.all(np.abs(X - x) <= (m + 1) * 4 * (np.log2(n) + 8) * eps * x)


@pytest.mark.parametrize("rounds", [1, 2])
@pytest.mark.parametrize("where", ["host", "device"])
def test_signed_fluid_folds_every_cycle(torch_cuda, where, rounds):
    """A right-hand side with negative entries runs the fold pass after each
    cycle (the kept-plus-pushed sum is not sum |F| for a signed fluid)."""
    torch = torch_cuda
    n = 10000
    src, dst = graphgen.web_graph(n, seed=9)
    rng = np.random.default_rng(12)
    B = rng.standard_normal(n) * 1e-4
    og = oracle.Graph(n, src, dst)
    X_ref, _, _ = oracle.diter(og, B, D, oracle.SOP, tol=1e-13)
    g = di.Graph(n, src, dst)
    pin_rounds(g, rounds)
    o = di.di_opts_default()
    o.kernel = WINDOW
    if where == "host":
        X, st = di.solve(g, B, D, TOL_PAR, kernel=WINDOW)
    else:
        Xd = torch.empty(n, dtype=torch.float64, device="cuda")
        status, st = di.di_solve_dev(g.handle, torch.from_numpy(B).cuda(), D, TOL_PAR, o, Xd)
        assert status == di.DI_OK, di.di_last_error()
        X = Xd.cpu().numpy()
        st = st.as_dict()
    assert np.abs(X - X_ref).sum() <= 1e-9
    _, r_true = oracle.residual(og, B, D, X)
    assert abs(r_true - st["resid_l1"]) <= 1e-14
    # and the selection follows the oracle cycle by cycle
    _, _, recs = traced(torch, g, B, 4096)
    check_against_oracle(og, g, B, recs)


def test_refined_and_fp32_window(torch_cuda):
    torch = torch_cuda
    n = 10000
    src, dst = graphgen.web_graph(n, seed=0)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    seeds = graphgen.ppr_seed_sets(n, 2)
    for j, S in enumerate(seeds):
        B = graphgen.ppr_rhs(n, S, D)
        X_ref, _, _ = oracle.diter(og, B, D, oracle.SOP, tol=1e-13)
        X, st = di.solve(g, B, D, 1e-9, kernel=WINDOW, precision=di.DI_FP32_REFINE)
        _, r_true = oracle.residual(og, B, D, X)
        assert r_true <= 1e-9, (j, r_true)
        assert np.abs(X - X_ref).sum() <= 1e-9 / (1 - D) + 1e-12
        assert st["refinements"] >= 1
    B = graphgen.uniform_rhs(n, D)
    X_ref, _, _ = oracle.diter(og, B, D, oracle.SOP, tol=1e-13)
    X, st = di.solve(g, None, D, 1e-7, kernel=WINDOW, precision=di.DI_FP32)
    assert np.abs(X - X_ref).sum() <= 2e-6 * X_ref.sum()


def test_paper_stop_and_max_cycles(torch_cuda):
    torch = torch_cuda
    n = 10000
    src, dst = graphgen.web_graph(n, seed=0)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    g = di.Graph(n, src, dst)
    # the paper's rule, target 1/N: the same stopping cycle as the oracle's
    # run in the same schedule, and the same estimate to rounding
    X, st = di.solve(g, None, D, 1.0 / n, kernel=WINDOW, stop=di.DI_STOP_PAPER)
    sch, kw = schedule_of(g, WINDOW)
    _, _, so = oracle.diter(og, B, D, oracle.SOP, sch, stop=oracle.STOP_PAPER, tol=1.0 / n, **kw)
    assert st["cycles"] == so.cycles
    assert abs(st["paper_err"] - so.paper_err) <= 1e-12 * so.paper_err
    # max_cycles: the history of exactly that many cycles (against the
    # oracle in the same schedule)
    for m in (1, 2, 9, 17):
        o = di.di_opts_default()
        o.kernel = WINDOW
        o.max_cycles = m
        Xw = torch.empty(n, dtype=torch.float64, device="cuda")
        status, stw = di.di_solve_dev(g.handle, None, D, 1e-15, o, Xw)
        assert status == di.DI_E_NOCONV and stw.cycles == m
        torch.cuda.synchronize()
        Ho, _, so = oracle.diter(og, B, D, oracle.SOP, sch, tol=0.0, max_cycles=m, **kw)
        assert so.cycles == m
        assert np.abs(Xw.cpu().numpy() - Ho).sum() <= 1e-13, m
        assert stw.edges_pushed == so.link_ops


def test_window_at_the_benchmark_configuration(torch_cuda):
    """N = 1M web graph, uniform B: every cycle's selection equals the
    oracle's synchronous cycle, X within 1e-9 of the oracle's solution, and
    the reported residual is the exact sum |F|."""
    n = 1_000_000
    src, dst = graphgen.web_graph(n, seed=0)
    B = graphgen.uniform_rhs(n, D)
    og = oracle.Graph(n, src, dst)
    g = di.Graph(n, src, dst)
    print("window 1M: traced solve", flush=True)
    X, st, recs = traced(torch_cuda, g, B, 4096)
    print(f"window 1M: {st.cycles} cycles; oracle cycles", flush=True)
    # r: the GPU tree sum and the oracle's sequential N-term sum differ by at
    # most (N - 1) u relative
    check_against_oracle(og, g, B, recs, rtol_r=(n - 1) * 2.0 ** -53)
    print("window 1M: oracle solve", flush=True)
    X_ref, _, _ = oracle.diter(og, B, D, oracle.SOP, tol=1e-13)
    assert np.abs(X - X_ref).sum() <= 1e-9
    _, r_true = oracle.residual(og, B, D, X)
    assert abs(r_true - st.resid_l1) <= 1e-14


def test_pinned_window_configuration(torch_cuda):
    """di_graph_set_window: out-of-range values are rejected with nothing
    changed; a pinned configuration is what DI_KERNEL_AUTO then runs (no
    tuning), including grids smaller than the tile count (blocks take
    several tiles) and one round a cycle (the synchronous schedule), and
    every one gives the oracle's cycles and solution and the exact
    residual."""
    n = 10000
    src, dst = graphgen.web_graph(n, seed=4)
    og = oracle.Graph(n, src, dst)
    B = graphgen.uniform_rhs(n, D)
    X_ref, _, _ = oracle.diter(og, B, D, oracle.SOP, tol=1e-13)
    g = di.Graph(n, src, dst)
    for bad in [(3000, 0, 8), (1024, -1, 8), (1024, 1025, 8), (1024, 0, 0), (1024, 0, 1025),
                (1024, 0, 8, 0), (1024, 0, 8, 3)]:
        assert di.di_graph_set_window(g.handle, *bad) == di.DI_E_INVAL, bad
    assert not di.di_graph_tuning(g.handle)["tuned"]
    for tile, hubs, grid, rounds in [(1024, 0, 3, 2), (1024, 64, 1024, 2), (2048, 64, 2, 2),
                                     (4096, 16, 1, 2), (2048, 64, 1024, 1)]:
        assert di.di_graph_set_window(g.handle, tile, hubs, grid, rounds) == di.DI_OK
        t = di.di_graph_tuning(g.handle)
        ntiles = (n + tile - 1) // tile
        assert t["kernel"] == "window" and t["tuned"]
        assert (t["tile"], t["hubs"], t["grid"], t["rounds"]) == (tile, hubs, min(grid, ntiles),
                                                                  rounds)
        print(f"pinned window: tile={tile} hubs={hubs} grid={grid} rounds={rounds}", flush=True)
        X, st = di.solve(g, None, D, TOL_PAR)
        assert np.abs(X - X_ref).sum() <= 1e-9, (tile, hubs, grid)
        _, r_true = oracle.residual(og, B, D, X)
        assert st["resid_l1"] <= TOL_PAR and abs(r_true - st["resid_l1"]) <= 1e-14
        # and the selections follow the oracle's synchronous cycles
        _, _, recs = traced(torch_cuda, g, B, 4096)
        check_against_oracle(og, g, B, recs)
