"""Pins of the oracle's paper-mode stop estimators and of its empty-cycle
fallback.

The paper stops each method on a normalized error estimate against the
target 1/N (Section 2.4):
  DI (Section 2.5.4):        sum F / (1 - d - d*e), e = fluid absorbed by
                             dangling nodes;
  GS (Section 2.5.3):        d * sum(x_new - x_old) / (1 - d - d*e), e = sum
                             of x over dangling nodes;
  PI, PI' (Sections 2.5.1-2): d/(1-d) * |x_new - x_old|_1 of the normalized
                             iterate.
Each is pinned by values derived by hand (tests/golden/) and by identities
that follow from conservation of fluid, evaluated here with dense matrices
rather than the oracle's own expression.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests._dense import dense_p

D = 0.85
HERE = os.path.dirname(os.path.abspath(__file__))


def _read(path):
    lines = [ln.split("#")[0].strip() for ln in open(path)]
    lines = [ln for ln in lines if ln]
    spec, runs, cur, step = {}, {}, None, None
    for ln in lines:
        key, *vals = ln.split()
        if key in ("schedule", "method"):
            cur = runs.setdefault(vals[0], [])
        elif key in ("cycle", "step"):
            step = {}
            cur.append(step)
        elif cur is None:
            spec[key] = vals
        elif key in ("selected", "link_ops"):
            step[key] = vals
        else:
            step[key] = [float(Fraction(v)) for v in vals]
    links = [tuple(int(x) for x in s.split(":")) for s in spec["links"]]
    src = np.array([a for a, _ in links], np.int32)
    dst = np.array([b for _, b in links], np.int32)
    return int(spec["n"][0]), float(Fraction(spec["d"][0])), src, dst, spec, runs


def test_di_paper_estimator_worked_example():
    """DI's estimator after each cycle of the hand-worked 4-node example,
    in both schedules."""
    n, d, src, dst, spec, runs = _read(os.path.join(HERE, "golden", "di_sop_worked_4node.txt"))
    B = np.array([float(Fraction(v)) for v in spec["B"]])
    g = oracle.Graph(n, src, dst)
    for sname, sch in (("sequential", oracle.SEQUENTIAL), ("sync", oracle.SYNC)):
        for c, want in enumerate(runs[sname], start=1):
            H, F, st = oracle.diter(g, B, d, oracle.SOP, sch, stop=oracle.STOP_PAPER, tol=0.0,
                                    max_cycles=c)
            assert st.cycles == c
            assert np.allclose(H, want["H"], rtol=0, atol=1e-16)
            assert abs(st.e - want["e"][0]) < 1e-16
            assert abs(st.paper_err - want["paper_err"][0]) <= 1e-15 * want["paper_err"][0], (
                sname, c, st.paper_err, want["paper_err"][0])


def test_gs_and_pi_paper_estimators_3node():
    """GS and PI / PI' estimators on the hand-worked 3-node graph with a
    dangling node."""
    n, d, src, dst, _, runs = _read(os.path.join(HERE, "golden", "paper_estimators_3node.txt"))
    g = oracle.Graph(n, src, dst)
    B = np.full(n, (1 - d) / n)
    for c, want in enumerate(runs["gs"], start=1):
        x, st = oracle.gs(g, B, d, stop=oracle.STOP_PAPER, tol=0.0, max_sweeps=c)
        assert st.cycles == c
        assert np.allclose(x, want["x"], rtol=0, atol=1e-16)
        assert abs(st.paper_err - want["paper_err"][0]) <= 1e-15 * want["paper_err"][0]
    for by_columns in (False, True):
        for c, want in enumerate(runs["pi"], start=1):
            x, st = oracle.pi(g, d, by_columns=by_columns, target=0.0, max_iter=c)
            assert st.cycles == c
            assert np.allclose(x, want["x"], rtol=0, atol=1e-16)
            assert abs(st.paper_err - want["paper_err"][0]) <= 2e-15 * want["paper_err"][0]


def _graph_with_dangling(rng, n):
    mask = rng.random((n, n)) < rng.uniform(0.08, 0.3)
    dang = rng.random(n) < 0.25
    dang[0] = True
    mask[dang, :] = False
    mask[~dang, 0] = True  # the dangling node 0 receives fluid
    src, dst = np.nonzero(mask)
    return src.astype(np.int32), dst.astype(np.int32)


@pytest.mark.parametrize("schedule", [oracle.SEQUENTIAL, oracle.SYNC])
@pytest.mark.parametrize("variant", [oracle.SOP, oracle.CYC])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_di_paper_estimator_conservation_identity(seed, variant, schedule):
    """With sum B = 1 - d, conservation of fluid (sum F = sum B - (1-d) sum H
    - d e) turns DI's normalizer into 1 - d - d*e = sum F + (1-d) sum H, so
    the estimator equals sum F / (sum F + (1-d) sum H) after every cycle."""
    rng = np.random.default_rng(100 + seed)
    n = 40
    src, dst = _graph_with_dangling(rng, n)
    g = oracle.Graph(n, src, dst)
    B = rng.random(n)
    B *= (1 - D) / B.sum()
    for c in range(1, 8):
        H, F, st = oracle.diter(g, B, D, variant, schedule, stop=oracle.STOP_PAPER, tol=0.0,
                                max_cycles=c)
        assert st.e > 0.0
        want = F.sum() / (F.sum() + (1 - D) * H.sum())
        assert abs(st.paper_err - want) <= 1e-12 * want, (c, st.paper_err, want)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gs_paper_estimator_residual_identity(seed):
    """For GS with sum B = 1 - d, summing R = B + P.x - x over the nodes gives
    1 - d - d*e = sum R + (1-d) sum x, with e = sum of x over dangling nodes;
    the sweep's increment is sum x_c - sum x_(c-1). R comes from a dense P."""
    rng = np.random.default_rng(200 + seed)
    n = 36
    src, dst = _graph_with_dangling(rng, n)
    g = oracle.Graph(n, src, dst)
    P = dense_p(n, src, dst, D)
    B = np.full(n, (1 - D) / n)
    prev = B.copy()
    for c in range(1, 6):
        x, st = oracle.gs(g, B, D, stop=oracle.STOP_PAPER, tol=0.0, max_sweeps=c)
        R = B + P @ x - x
        want = D * (x.sum() - prev.sum()) / (R.sum() + (1 - D) * x.sum())
        assert abs(st.paper_err - want) <= 1e-9 * abs(want), (c, st.paper_err, want)
        prev = x


@pytest.mark.parametrize("by_columns", [False, True])
def test_pi_iterates_and_estimator_against_dense_powers(by_columns):
    """PI's renormalized step is x <- M x with M = P + (1/N) 1 (1^T (I - P))
    (for sum x = 1); the iterates from 1/N are powers of M, and the estimator
    is d/(1-d) times the L1 step between consecutive powers."""
    rng = np.random.default_rng(7)
    n = 30
    src, dst = _graph_with_dangling(rng, n)
    g = oracle.Graph(n, src, dst)
    P = dense_p(n, src, dst, D)
    M = P + np.outer(np.ones(n), np.ones(n) @ (np.eye(n) - P)) / n
    xs = [np.full(n, 1.0 / n)]
    for c in range(1, 7):
        xs.append(M @ xs[-1])
        x, st = oracle.pi(g, D, by_columns=by_columns, target=0.0, max_iter=c)
        assert np.abs(x - xs[c]).sum() < 1e-14
        want = D / (1 - D) * np.abs(xs[c] - xs[c - 1]).sum()
        assert abs(st.paper_err - want) <= 1e-10 * want, (c, st.paper_err, want)


def test_empty_sop_cycle_falls_back_to_one_cyc_cycle():
    """On the directed 3-cycle with B = 0.1 everywhere, r = 0.1 + 0.1 + 0.1
    rounds to 0.30000000000000004 and r/L * 1 to 0.10000000000000002, above
    every F_i: the DI-SOP rule selects nothing, so one DI-CYC cycle follows.
    The solution is the closed form X_i = B_i / (1 - d)."""
    assert (0.1 + 0.1 + 0.1) / 3 * 1 > 0.1  # the IEEE rounding the case relies on
    n = 3
    src = np.array([0, 1, 2], np.int32)
    dst = np.array([1, 2, 0], np.int32)
    g = oracle.Graph(n, src, dst)
    B = np.full(n, 0.1)
    F, H = B.copy(), np.zeros(n)
    cnt, sel, e, ops, r = oracle.di_cycle(g, F, H, D, oracle.SOP, oracle.SYNC)
    assert cnt == 0 and ops == 0 and not sel.any()
    for sch in (oracle.SEQUENTIAL, oracle.SYNC):
        H, F, st = oracle.diter(g, B, D, oracle.SOP, sch, tol=1e-13)
        assert st.status == oracle.OK
        assert st.fallback_cycles >= 1
        assert np.abs(H - B / (1 - D)).sum() <= 1e-13 / (1 - D) + 1e-15
        # the first cycle alone: the empty DI-SOP cycle and its DI-CYC cycle
        H1, F1, st1 = oracle.diter(g, B, D, oracle.SOP, sch, tol=0.0, max_cycles=1)
        assert st1.fallback_cycles == 1
        assert st1.link_ops == 3
        # sync: every node diffuses its 0.1; sequential: node 1 already
        # holds 0.1 + 0.85*0.1 when its turn comes, node 2 0.1 + 0.85*0.185
        want = [0.1, 0.1, 0.1] if sch == oracle.SYNC else [0.1, 0.185, 0.25725]
        assert np.allclose(H1, want, rtol=0, atol=1e-16)
