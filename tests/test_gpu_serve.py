"""GPU tests of the serving loop (continuous batching of personalized
PageRank requests) through the C ABI.

Every finished request is checked against the CPU oracle: its residual,
recomputed by the oracle, must be within its tolerance, and its distance to
the oracle's solution within tol / (1 - d) (the residual bound: P's columns
sum to at most d) plus 1e-12. A
request served alone and the same request served in a mix of others must
both pass; they may differ only within those bounds.
"""

import threading
import time

import numpy as np
import pytest

import oracle
from paper_1204_6255_amd import di, graphgen

pytestmark = pytest.mark.gpu

D = 0.85
GIB = 1 << 30


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


_GRAPHS = {}


def graph(n, seed):
    key = (n, seed)
    if key not in _GRAPHS:
        src, dst = graphgen.web_graph(n, seed=seed)
        _GRAPHS[key] = (src, dst, di.Graph(n, src, dst), oracle.Graph(n, src, dst))
    return _GRAPHS[key]


class Server:
    def __init__(self, budget, k_max, opts=None):
        st, self.h = di.di_serve_create(budget, k_max, opts)
        assert st == di.DI_OK, di.di_last_error()

    def close(self):
        if self.h:
            di.di_serve_destroy(self.h)
            self.h = None


def wait(srv, ticket, n, timeout=120.0):
    X = np.empty(n)
    t0 = time.time()
    while True:
        st, stats = di.di_serve_poll(srv.h, ticket, X)
        if st != di.DI_PENDING:
            return st, X, stats
        assert time.time() - t0 < timeout, "request did not finish"
        time.sleep(0.0005)


def check(og, seeds, tol, X):
    n = og.n
    B = graphgen.ppr_rhs(n, seeds, D) if len(seeds) else graphgen.uniform_rhs(n, D)
    ref, _, st = oracle.diter(og, B, D, oracle.SOP, oracle.SEQUENTIAL, tol=1e-13)
    _, r = oracle.residual(og, B, D, X)
    assert r <= tol * (1 + 1e-6) + 1e-16
    assert np.abs(X - ref).sum() <= tol / (1 - D) + 1e-12


def test_alone_and_in_a_mix(torch_cuda):
    _, _, g1, og1 = graph(10000, 0)
    _, _, g2, og2 = graph(20000, 1)
    seeds = graphgen.ppr_seed_sets(10000, 1, 4242)[0]
    # alone
    srv = Server(8 * GIB, 16)
    assert di.di_serve_add_graph(srv.h, g1.handle, 1) == di.DI_OK
    st, t = di.di_serve_submit(srv.h, 1, seeds, D, 1e-9)
    assert st == di.DI_OK
    st, X_alone, s_alone = wait(srv, t, 10000)
    assert st == di.DI_OK, di.di_last_error()
    srv.close()
    check(og1, seeds, 1e-9, X_alone)
    # in a mix: two graphs, other seed sets and tolerances, submitted around it
    srv = Server(8 * GIB, 16)
    assert di.di_serve_add_graph(srv.h, g1.handle, 1) == di.DI_OK
    assert di.di_serve_add_graph(srv.h, g2.handle, 2) == di.DI_OK
    others = []
    for j, s in enumerate(graphgen.ppr_seed_sets(20000, 12, 77)):
        st, tk = di.di_serve_submit(srv.h, 2, s, D, 1e-6 if j % 2 else 1e-9)
        assert st == di.DI_OK
        others.append((og2, s, 1e-6 if j % 2 else 1e-9, tk, 20000))
    for j, s in enumerate(graphgen.ppr_seed_sets(10000, 6, 99)):
        st, tk = di.di_serve_submit(srv.h, 1, s, D, 1e-6)
        others.append((og1, s, 1e-6, tk, 10000))
    st, t = di.di_serve_submit(srv.h, 1, seeds, D, 1e-9)
    st, X_mix, s_mix = wait(srv, t, 10000)
    assert st == di.DI_OK
    check(og1, seeds, 1e-9, X_mix)
    assert np.abs(X_mix - X_alone).sum() <= 2e-9 / (1 - D)
    for og, s, tol, tk, n in others:
        st, X, _ = wait(srv, tk, n)
        assert st == di.DI_OK
        check(og, s, tol, X)
    _, info = di.di_serve_info(srv.h)
    assert info.completed == info.submitted == 19 and info.active == 0 and info.pending == 0
    srv.close()


def test_more_requests_than_columns(torch_cuda):
    """30 requests through 8 columns: columns are reused as requests finish."""
    _, _, g, og = graph(10000, 0)
    srv = Server(8 * GIB, 8)
    assert di.di_serve_add_graph(srv.h, g.handle, 0) == di.DI_OK
    sets = graphgen.ppr_seed_sets(10000, 30, 500)
    tickets = []
    for j, s in enumerate(sets):
        st, tk = di.di_serve_submit(srv.h, 0, s, D, 1e-9 if j % 3 else 1e-6)
        assert st == di.DI_OK
        tickets.append(tk)
    for j, (s, tk) in enumerate(zip(sets, tickets)):
        st, X, stats = wait(srv, tk, 10000)
        assert st == di.DI_OK
        if j % 5 == 0:
            check(og, s, 1e-9 if j % 3 else 1e-6, X)
        assert stats.seconds > 0 and stats.cycles > 0
    srv.close()


def test_uniform_request_is_pagerank(torch_cuda):
    _, _, g, og = graph(10000, 0)
    srv = Server(8 * GIB, 8, None)
    di.di_serve_add_graph(srv.h, g.handle, 5)
    st, tk = di.di_serve_submit(srv.h, 5, None, D, 1.4e-10)
    st, X, _ = wait(srv, tk, 10000)
    assert st == di.DI_OK
    check(og, [], 1.4e-10, X)
    srv.close()


def test_admission_by_hbm_budget(torch_cuda):
    """A budget that holds one graph's batch at a time: the second graph's
    requests wait for the first batch to go idle (admission stalls), and
    every request still finishes correctly."""
    _, _, g1, og1 = graph(10000, 0)
    _, _, g2, og2 = graph(20000, 1)
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    o.flags = di.DI_FLAG_SERVE_NO_SOLO  # column sets only: their admission is tested
    # batch bytes of the larger graph, plus a little: never both at once
    # (KP = 8: 3 float arrays + 3 double arrays of n * 8, plus small records)
    budget = 20000 * 8 * (3 * 4 + 3 * 8) + 20000 * 8 + (1 << 20)
    srv = Server(budget, 8, o)
    assert di.di_serve_add_graph(srv.h, g1.handle, 1) == di.DI_OK
    assert di.di_serve_add_graph(srv.h, g2.handle, 2) == di.DI_OK
    reqs = []
    for j in range(10):
        gid, og, n = (1, og1, 10000) if j % 2 == 0 else (2, og2, 20000)
        s = graphgen.ppr_seed_sets(n, 1, 3000 + j)[0]
        st, tk = di.di_serve_submit(srv.h, gid, s, D, 1e-9)
        assert st == di.DI_OK
        reqs.append((og, s, tk, n))
    for og, s, tk, n in reqs:
        st, X, _ = wait(srv, tk, n)
        assert st == di.DI_OK
        check(og, s, 1e-9, X)
    _, info = di.di_serve_info(srv.h)
    assert info.admission_stalls >= 1
    assert info.bytes_in_use <= budget
    srv.close()


def test_lone_request_runs_solo(torch_cuda):
    """A request alone on its graph takes the single right-hand side path in
    FP64 (no residual passes, whatever the server's precision); with
    DI_FLAG_SERVE_NO_SOLO it runs in a column set. Both meet the bar, and a
    solo request and column sets on the same graph overlap correctly."""
    _, _, g, og = graph(10000, 0)
    seeds = graphgen.ppr_seed_sets(10000, 1, 4243)[0]
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    o.kernel = di.DI_KERNEL_PULL  # solo slots on the select + pull pair
    srv = Server(8 * GIB, 16, o)
    assert di.di_serve_add_graph(srv.h, g.handle, 0) == di.DI_OK
    st, t = di.di_serve_submit(srv.h, 0, seeds, D, 1e-9)
    st, X_solo, s_solo = wait(srv, t, 10000)
    assert st == di.DI_OK, di.di_last_error()
    check(og, seeds, 1e-9, X_solo)
    assert s_solo.refinements == 0 and s_solo.cycles > 0 and s_solo.seconds > 0
    # the same request's FP64 single solve gives the same cycles
    B = graphgen.ppr_rhs(10000, seeds, D)
    X1 = np.empty(10000)
    o1 = di.di_opts_default()
    o1.kernel = di.DI_KERNEL_PULL
    status, st1 = di.di_solve(g.handle, B, D, 1e-9, o1, X1)
    assert status == di.DI_OK and st1.cycles == s_solo.cycles
    assert np.array_equal(X1, X_solo)  # same kernels, deterministic pull
    # uniform B through the solo slot
    st, t = di.di_serve_submit(srv.h, 0, None, D, 1.4e-10)
    st, Xu, su = wait(srv, t, 10000)
    assert st == di.DI_OK and su.refinements == 0
    check(og, [], 1.4e-10, Xu)
    # a solo request, then a burst on the same graph while it runs
    reqs = [(seeds, 1e-9)] + [(s, 1e-6 if j % 2 else 1e-9)
                              for j, s in enumerate(graphgen.ppr_seed_sets(10000, 9, 600))]
    tickets = []
    for s_, tol in reqs:
        st, tk = di.di_serve_submit(srv.h, 0, s_, D, tol)
        assert st == di.DI_OK
        tickets.append(tk)
    for (s_, tol), tk in zip(reqs, tickets):
        st, X, _ = wait(srv, tk, 10000)
        assert st == di.DI_OK
        check(og, s_, tol, X)
    _, info = di.di_serve_info(srv.h)
    assert info.completed == info.submitted == 12 and info.active == 0 and info.pending == 0
    srv.close()
    # the same lone request in a column set
    o.flags = di.DI_FLAG_SERVE_NO_SOLO
    srv = Server(8 * GIB, 16, o)
    assert di.di_serve_add_graph(srv.h, g.handle, 0) == di.DI_OK
    st, t = di.di_serve_submit(srv.h, 0, seeds, D, 1e-9)
    st, X_set, s_set = wait(srv, t, 10000)
    assert st == di.DI_OK
    check(og, seeds, 1e-9, X_set)
    assert s_set.refinements >= 1
    assert np.abs(X_set - X_solo).sum() <= 2e-9 / (1 - D)
    srv.close()


def test_solo_slots_at_light_load(torch_cuda):
    """A few requests at once on one graph all run in solo slots (FP64, no
    residual passes; DI-SOP on the graph's tuned kernel, tuned when the graph
    is registered), two of them after waiting for a free slot; a burst past
    twice the slots also fills column sets. Every request meets the bar, and
    its latency splits exactly into waiting, running and reading out."""
    _, _, g, og = graph(20000, 3)
    srv = Server(8 * GIB, 16)
    assert di.di_serve_add_graph(srv.h, g.handle, 0) == di.DI_OK
    tun = di.di_graph_tuning(g.handle)
    assert tun["tuned"] and tun["kernel"] in ("window", "pull")
    seeds = graphgen.ppr_seed_sets(20000, 6, 777)
    tickets = []
    for j, s_ in enumerate(seeds):
        st, tk = di.di_serve_submit(srv.h, 0, s_, D, 1e-9 if j % 2 else 1e-7)
        assert st == di.DI_OK
        tickets.append(tk)
    for j, (s_, tk) in enumerate(zip(seeds, tickets)):
        st, X, sts = wait(srv, tk, 20000)
        assert st == di.DI_OK, di.di_last_error()
        check(og, s_, 1e-9 if j % 2 else 1e-7, X)
        assert sts.refinements == 0 and sts.cycles > 0
        assert sts.queue_seconds >= 0 and sts.run_seconds > 0 and sts.readout_seconds >= 0
        total = sts.queue_seconds + sts.run_seconds + sts.readout_seconds
        assert abs(total - sts.seconds) <= 1e-9
    _, info = di.di_serve_info(srv.h)
    assert info.solo_requests == 6 and info.completed == 6
    # a burst of 20: past twice the solo slots, column sets take the rest
    burst = graphgen.ppr_seed_sets(20000, 20, 778)
    tickets = [di.di_serve_submit(srv.h, 0, s_, D, 1e-8)[1] for s_ in burst]
    for s_, tk in zip(burst, tickets):
        st, X, sts = wait(srv, tk, 20000)
        assert st == di.DI_OK
        check(og, s_, 1e-8, X)
    _, info = di.di_serve_info(srv.h)
    assert info.completed == 26 and 6 <= info.solo_requests < 26
    assert info.active == 0 and info.pending == 0
    srv.close()


def test_concurrent_submitters(torch_cuda):
    _, _, g, og = graph(10000, 0)
    srv = Server(8 * GIB, 32)
    di.di_serve_add_graph(srv.h, g.handle, 0)
    out = {}
    errors = []

    def client(cid):
        try:
            for j, s in enumerate(graphgen.ppr_seed_sets(10000, 5, 9000 + 10 * cid)):
                st, tk = di.di_serve_submit(srv.h, 0, s, D, 1e-8)
                assert st == di.DI_OK
                st, X, _ = wait(srv, tk, 10000)
                assert st == di.DI_OK
                out[(cid, j)] = (s, X)
        except AssertionError as e:  # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert not errors and len(out) == 20
    for key in [(0, 0), (3, 4)]:
        s, X = out[key]
        check(og, s, 1e-8, X)
    srv.close()


def test_serving_errors(torch_cuda):
    _, _, g, og = graph(10000, 0)
    st, h = di.di_serve_create(GIB, 0)
    assert st == di.DI_E_INVAL
    st, h = di.di_serve_create(GIB, 300)
    assert st == di.DI_E_INVAL
    srv = Server(GIB, 8)
    assert di.di_serve_add_graph(srv.h, g.handle, 3) == di.DI_OK
    assert di.di_serve_add_graph(srv.h, g.handle, 3) == di.DI_E_INVAL
    st, _ = di.di_serve_submit(srv.h, 4, [1, 2], D, 1e-9)
    assert st == di.DI_E_NOTFOUND
    st, _ = di.di_serve_submit(srv.h, 3, [1, 10000], D, 1e-9)
    assert st == di.DI_E_RANGE
    st, _ = di.di_serve_submit(srv.h, 3, [1], 1.0, 1e-9)
    assert st == di.DI_E_INVAL
    st, _ = di.di_serve_submit(srv.h, 3, [1], D, 0.0)
    assert st == di.DI_E_INVAL
    st, _ = di.di_serve_poll(srv.h, 12345)
    assert st == di.DI_E_NOTFOUND
    # a collected ticket is forgotten; duplicate seeds count once
    st, tk = di.di_serve_submit(srv.h, 3, [5, 5, 17], D, 1e-9)
    st, X, _ = wait(srv, tk, 10000)
    assert st == di.DI_OK
    check(og, [5, 17], 1e-9, X)
    st, _ = di.di_serve_poll(srv.h, tk)
    assert st == di.DI_E_NOTFOUND
    # a graph whose batch exceeds the budget is refused
    small = Server(1 << 20, 8)
    assert di.di_serve_add_graph(small.h, g.handle, 0) == di.DI_E_NOMEM
    small.close()
    srv.close()


def test_all_nodes_seed_set_is_uniform_pagerank(torch_cuda):
    """A seed set of every node gives B = (1-d)/N, the uniform right-hand
    side: served alone and in a column set, the answer equals the uniform
    request's (bit for bit on the deterministic paths: the solo slot's pull
    and the column sets; to rounding on the solo slot's tuned kernel, whose
    window push adds far links in a varying order), and a batch column with
    that B equals a uniform column."""
    n = 10000
    _, _, g, og = graph(n, 0)
    every = np.arange(n, dtype=np.int32)
    for flags, kernel in ((0, di.DI_KERNEL_PULL), (0, di.DI_KERNEL_AUTO),
                          (di.DI_FLAG_SERVE_NO_SOLO, di.DI_KERNEL_AUTO)):
        o = di.di_opts_default()
        o.precision = di.DI_FP32_REFINE
        o.flags = flags
        o.kernel = kernel
        srv = Server(8 * GIB, 8, o)
        di.di_serve_add_graph(srv.h, g.handle, 0)
        st, t1 = di.di_serve_submit(srv.h, 0, every, D, 1e-9)
        st, X1, _ = wait(srv, t1, n)
        assert st == di.DI_OK
        st, t2 = di.di_serve_submit(srv.h, 0, None, D, 1e-9)
        st, X2, _ = wait(srv, t2, n)
        assert st == di.DI_OK
        check(og, [], 1e-9, X1)
        check(og, [], 1e-9, X2)
        if flags or kernel == di.DI_KERNEL_PULL or di.di_graph_tuning(g.handle)["kernel"] == "pull":
            assert np.array_equal(X1, X2)
        else:
            assert np.abs(X1 - X2).sum() <= 1e-12
        srv.close()
    B = np.stack([graphgen.ppr_rhs(n, every, D), graphgen.uniform_rhs(n, D)])
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE
    status, Xb, _ = di.di_solve_batch(g.handle, 2, B, D, [1e-9, 1e-9], o)
    assert status == di.DI_OK
    assert np.array_equal(Xb[0], Xb[1])
