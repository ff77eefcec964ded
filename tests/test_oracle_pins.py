"""Pins of the CPU oracle against what the mathematics fixes.

Each check uses something other than the oracle's own code: dense Gaussian
elimination of (I - P) X = B, closed forms, a hand-worked example, brute
force over every 3-node digraph, and invariants of the D-iteration update.
"""

import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests._dense import dense_p, dense_solve

D = 0.85
HERE = os.path.dirname(os.path.abspath(__file__))
# the D-iteration schedules: the paper's sequential cycle, the
# frontier-synchronous one, and tiled ones (two and three rounds a cycle)
SCHEDULES = [("seq", oracle.SEQUENTIAL, {}), ("sync", oracle.SYNC, {}),
             ("tiled-4-2", oracle.TILED, dict(tile=4, reach=2, rounds=2)),
             ("tiled-16-5", oracle.TILED, dict(tile=16, reach=5, rounds=3))]


def _all_methods(g, B, d, tol):
    """Every oracle solve of the unnormalized system, tagged."""
    out = {}
    for var, vname in ((oracle.SOP, "sop"), (oracle.CYC, "cyc")):
        for sname, sch, kw in SCHEDULES:
            H, F, st = oracle.diter(g, B, d, var, sch, tol=tol, **kw)
            assert st.status == oracle.OK
            out[f"di-{vname}-{sname}"] = (H, st)
    x, st = oracle.gs(g, B, d, tol=tol)
    assert st.status == oracle.OK
    out["gs"] = (x, st)
    x, st = oracle.jacobi(g, B, d, tol=tol)
    assert st.status == oracle.OK
    out["jacobi"] = (x, st)
    return out


def _random_graph(rng, n):
    """Random digraph with dangling nodes, self-loops, isolated nodes and a
    zero in-degree chain."""
    p = rng.uniform(0.05, 0.4)
    mask = rng.random((n, n)) < p
    dang = rng.random(n) < 0.2
    mask[dang, :] = False  # dangling rows (no out-links)
    if n >= 6:
        iso = rng.integers(0, n)
        mask[iso, :] = False
        mask[:, iso] = False
        # chain a -> b -> c where a has no in-links
        a, b, c = rng.choice(n, 3, replace=False)
        mask[:, a] = False
        mask[a, b] = True
        mask[b, c] = True
    src, dst = np.nonzero(mask)
    return src.astype(np.int32), dst.astype(np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_all_methods_match_dense_solve(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 51))
    src, dst = _random_graph(rng, n)
    B = rng.random(n) * (rng.random(n) < 0.7)
    if B.sum() == 0:
        B[0] = 1.0
    X, _ = dense_solve(n, src, dst, D, B)
    g = oracle.Graph(n, src, dst)
    tol = 1e-13 * max(B.sum(), 1.0)
    for name, (x, st) in _all_methods(g, B, D, tol).items():
        err = np.abs(x - X).sum()
        assert err <= tol / (1 - D) + 1e-13 * X.sum(), (name, err)


def test_brute_force_every_3_node_digraph():
    n = 3
    pairs = [(i, j) for i in range(n) for j in range(n)]
    B = np.array([0.3, 0.05, 0.11])
    tol = 1e-14
    for bits in range(1 << 9):
        links = [pairs[k] for k in range(9) if bits >> k & 1]
        src = np.array([a for a, _ in links], dtype=np.int32)
        dst = np.array([b for _, b in links], dtype=np.int32)
        X, _ = dense_solve(n, src, dst, D, B)
        g = oracle.Graph(n, src, dst)
        for name, (x, st) in _all_methods(g, B, D, tol).items():
            assert np.abs(x - X).sum() <= tol / (1 - D) + 1e-14, (bits, name)


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_closed_form_directed_cycle(n):
    src = np.arange(n, dtype=np.int32)
    dst = ((np.arange(n) + 1) % n).astype(np.int32)
    g = oracle.Graph(n, src, dst)
    B = np.full(n, (1 - D) / n)
    for name, (x, _) in _all_methods(g, B, D, 1e-14).items():
        # n = 1 is a lone self-loop: X = B/(1-d) = 1 as well
        assert np.allclose(x, 1.0 / n, rtol=0, atol=1e-13), name


@pytest.mark.parametrize("loops", [False, True])
@pytest.mark.parametrize("n", [2, 5, 23])
def test_closed_form_complete_digraph(n, loops):
    pairs = [(i, j) for i in range(n) for j in range(n) if loops or i != j]
    src = np.array([a for a, _ in pairs], dtype=np.int32)
    dst = np.array([b for _, b in pairs], dtype=np.int32)
    g = oracle.Graph(n, src, dst)
    B = np.full(n, (1 - D) / n)
    for name, (x, _) in _all_methods(g, B, D, 1e-14).items():
        assert np.allclose(x, 1.0 / n, rtol=0, atol=1e-13), name


def test_closed_form_self_loop_only_node():
    # node 0: only a self-loop (p_00 = d); node 1: isolated and dangling
    g = oracle.Graph(2, np.array([0], np.int32), np.array([0], np.int32))
    B = np.array([0.2, 0.3])
    for name, (x, _) in _all_methods(g, B, D, 1e-15).items():
        assert abs(x[0] - 0.2 / (1 - D)) < 1e-13, name
        assert abs(x[1] - 0.3) < 1e-15, name
    # D-iteration clears it in one diffusion through the transit formula
    H, F, st = oracle.diter(g, B, D, oracle.CYC, tol=0.0)
    assert st.cycles == 1 and np.all(F == 0.0)


def test_closed_form_chain_and_dip_sop_tie():
    """0 -> 1, uniform B: X = ((1-d)/2, (1-d)(1+d)/2). With a strict '>'
    DI-SOP would stall here (F_0 equals its threshold r*1/1 forever once
    node 1 is empty); the '>=' reading converges with no fallback."""
    g = oracle.Graph(2, np.array([0], np.int32), np.array([1], np.int32))
    B = np.full(2, (1 - D) / 2)
    expect = np.array([(1 - D) / 2, (1 - D) * (1 + D) / 2])
    H, F, st = oracle.diter(g, B, D, oracle.SOP, tol=0.0, max_cycles=10)
    assert st.status == oracle.OK
    assert st.fallback_cycles == 0
    assert np.all(F == 0.0)
    assert np.allclose(H, expect, rtol=0, atol=1e-16)
    for name, (x, _) in _all_methods(g, B, D, 1e-15).items():
        assert np.allclose(x, expect, rtol=0, atol=1e-15), name


def test_closed_form_no_links():
    g = oracle.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    B = np.array([0.1, 0.0, 0.2, 0.3, 0.4])
    H, F, st = oracle.diter(g, B, D, oracle.SOP, tol=0.0)
    assert np.array_equal(H, B) and st.cycles == 1 and st.link_ops == 0
    for name, (x, _) in _all_methods(g, B, D, 0.0).items():
        assert np.array_equal(x, B), name


def test_dag_in_topological_order_is_exact_after_one_pass():
    """Zero in-degree nodes (E of Section 2.4) converge in finite steps: on a
    DAG numbered in topological order, one DI-CYC cycle leaves no fluid and
    one GS sweep is exact."""
    rng = np.random.default_rng(7)
    n = 30
    mask = np.triu(rng.random((n, n)) < 0.3, k=1)
    src, dst = np.nonzero(mask)
    src, dst = src.astype(np.int32), dst.astype(np.int32)
    B = rng.random(n)
    X, _ = dense_solve(n, src, dst, D, B)
    g = oracle.Graph(n, src, dst)
    H, F, st = oracle.diter(g, B, D, oracle.CYC, tol=0.0, max_cycles=5)
    assert st.cycles == 1 and np.all(F == 0.0)
    assert np.abs(H - X).sum() <= 1e-14 * X.sum()
    x, st = oracle.gs(g, B, D, tol=1e-14 * X.sum())
    assert st.cycles == 1
    assert np.abs(x - X).sum() <= 1e-14 * X.sum()


def _read_worked_example():
    path = os.path.join(HERE, "golden", "di_sop_worked_4node.txt")
    lines = [ln.split("#")[0].strip() for ln in open(path)]
    lines = [ln for ln in lines if ln]
    spec, runs, cur, cyc = {}, {}, None, None
    for ln in lines:
        key, *vals = ln.split()
        if key == "schedule":
            cur = runs.setdefault(vals[0], [])
        elif key == "cycle":
            cyc = {}
            cur.append(cyc)
        elif cur is None:
            spec[key] = vals
        elif key in ("selected",):
            cyc[key] = [int(v) for v in vals]
        elif key == "link_ops":
            cyc[key] = int(vals[0])
        else:
            cyc[key] = [float(Fraction(v)) for v in vals]
    return spec, runs


def test_worked_example_selection_and_update():
    """Hand-worked DI-SOP cycles (tests/golden/di_sop_worked_4node.txt)."""
    spec, runs = _read_worked_example()
    n = int(spec["n"][0])
    d = float(Fraction(spec["d"][0]))
    links = [tuple(int(x) for x in s.split(":")) for s in spec["links"]]
    src = np.array([a for a, _ in links], np.int32)
    dst = np.array([b for _, b in links], np.int32)
    B = np.array([float(Fraction(v)) for v in spec["B"]])
    g = oracle.Graph(n, src, dst)
    for sname, sch in (("sequential", oracle.SEQUENTIAL), ("sync", oracle.SYNC)):
        F = B.copy()
        H = np.zeros(n)
        e = 0.0
        for c in runs[sname]:
            cnt, sel, e, ops, r = oracle.di_cycle(g, F, H, d, oracle.SOP, sch, e)
            assert list(np.nonzero(sel)[0]) == c["selected"], (sname, c)
            assert cnt == len(c["selected"])
            assert ops == c["link_ops"]
            assert abs(r - c["r"][0]) < 1e-16
            assert np.allclose(F, c["F"], rtol=0, atol=1e-16), (sname, F, c["F"])
            assert np.allclose(H, c["H"], rtol=0, atol=1e-16), (sname, H, c["H"])
            assert abs(e - c["e"][0]) < 1e-16


@pytest.mark.parametrize("sname,schedule,kw", SCHEDULES[:3])
@pytest.mark.parametrize("variant", [oracle.SOP, oracle.CYC])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants_every_cycle(seed, variant, sname, schedule, kw):
    """F_n = B - (I-P) H_n; conservation of fluid; |F|_1 non-increasing and H
    non-decreasing for B >= 0; H_n + (I-P)^-1 F_n = X; and the stopping
    bound |X - H_n|_1 <= |F_n|_1 / (1-d)."""
    rng = np.random.default_rng(100 + seed)
    n = 45
    src, dst = _random_graph(rng, n)
    B = rng.random(n)
    X, P = dense_solve(n, src, dst, D, B)
    A = np.eye(n) - P
    out = np.bincount(src, minlength=n)
    g = oracle.Graph(n, src, dst)
    F = B.copy()
    H = np.zeros(n)
    e = 0.0
    prev_l1 = F.sum()
    for _ in range(25):
        prev_H = H.copy()
        _, _, e, _, _ = oracle.di_cycle(g, F, H, D, variant, schedule, e, **kw)
        assert np.abs(F - (B - A @ H)).sum() <= 1e-14 * B.sum()
        cons = F.sum() + (1 - D) * H[out > 0].sum() + H[out == 0].sum()
        assert abs(cons - B.sum()) <= 1e-14 * B.sum()
        assert F.min() >= 0.0
        assert F.sum() <= prev_l1 * (1 + 1e-15)
        assert np.all(H >= prev_H)
        prev_l1 = F.sum()
        assert np.abs(H + np.linalg.solve(A, F) - X).sum() <= 1e-13 * X.sum()
        assert np.abs(X - H).sum() <= F.sum() / (1 - D) + 1e-14 * X.sum()


def test_absorbed_mass_e_matches_dangling_history():
    rng = np.random.default_rng(5)
    n = 40
    src, dst = _random_graph(rng, n)
    out = np.bincount(src, minlength=n)
    B = rng.random(n)
    g = oracle.Graph(n, src, dst)
    H, F, st = oracle.diter(g, B, D, oracle.SOP, tol=1e-12)
    assert abs(st.e - H[out == 0].sum()) <= 1e-14 * B.sum()


def test_link_ops_count_excludes_self_loops():
    """A DI-CYC cycle from B > 0 diffuses every node: the link operations are
    the links minus the self-loops."""
    rng = np.random.default_rng(11)
    n = 30
    src, dst = _random_graph(rng, n)
    g = oracle.Graph(n, src, dst)
    F = rng.random(n) + 0.1
    H = np.zeros(n)
    cnt, sel, e, ops, r = oracle.di_cycle(g, F, H, D, oracle.CYC, oracle.SYNC)
    assert cnt == n
    assert ops == int(np.sum(src != dst))


def test_residual_and_apply_p_against_dense():
    rng = np.random.default_rng(3)
    n = 37
    src, dst = _random_graph(rng, n)
    P = dense_p(n, src, dst, D)
    g = oracle.Graph(n, src, dst)
    B = rng.random(n)
    X = rng.standard_normal(n)
    R, l1 = oracle.residual(g, B, D, X)
    assert np.allclose(R, B + P @ X - X, rtol=0, atol=1e-14)
    assert abs(l1 - np.abs(B + P @ X - X).sum()) < 1e-13
    assert np.allclose(oracle.apply_p(g, D, X), P @ X, rtol=0, atol=1e-14)


@pytest.mark.parametrize("by_columns", [False, True])
def test_power_iteration_is_normalized_solution(by_columns):
    """PI and PI' renormalize every step; their fixed point is X/|X|_1 for the
    uniform B, dangling nodes included."""
    rng = np.random.default_rng(21)
    n = 48
    src, dst = _random_graph(rng, n)
    B = np.full(n, (1 - D) / n)
    X, _ = dense_solve(n, src, dst, D, B)
    g = oracle.Graph(n, src, dst)
    x, st = oracle.pi(g, D, by_columns=by_columns, target=1e-14)
    assert st.status == oracle.OK
    assert np.abs(x - X / X.sum()).sum() < 1e-12
    assert abs(x.sum() - 1.0) < 1e-13


def test_paper_mode_estimators_bound_the_relative_error():
    """The paper's stopping rules (target 1/N) estimate the relative L1 error
    of the normalized vector; at their stop the true relative error is below
    a small multiple of the target."""
    rng = np.random.default_rng(8)
    n = 50
    src, dst = _random_graph(rng, n)
    B = np.full(n, (1 - D) / n)
    X, _ = dense_solve(n, src, dst, D, B)
    xn = X / X.sum()
    g = oracle.Graph(n, src, dst)
    target = 1.0 / n
    H, F, st = oracle.diter(g, B, D, oracle.SOP, stop=oracle.STOP_PAPER, tol=target)
    assert st.paper_err <= target
    assert np.abs(H / H.sum() - xn).sum() <= 2 * target
    x, st = oracle.gs(g, B, D, stop=oracle.STOP_PAPER, tol=target)
    assert st.paper_err <= target
    assert np.abs(x / x.sum() - xn).sum() <= 2 * target
    x, st = oracle.pi(g, D, target=target)
    assert np.abs(x - xn).sum() <= 2 * target


def test_linearity_in_b():
    rng = np.random.default_rng(4)
    n = 44
    src, dst = _random_graph(rng, n)
    g = oracle.Graph(n, src, dst)
    Bs = [rng.random(n) for _ in range(3)]
    a = np.array([0.5, 2.0, 0.25])
    tol = 1e-14
    xs = [oracle.diter(g, b, D, tol=tol)[0] for b in Bs]
    x_mix = oracle.diter(g, sum(ai * b for ai, b in zip(a, Bs)), D, tol=tol)[0]
    assert np.abs(x_mix - sum(ai * x for ai, x in zip(a, xs))).sum() < 1e-12


def test_signed_right_hand_side():
    """A residual used as a right-hand side can be negative; |F| drives the
    selection and every method still reaches (I-P)^-1 B."""
    rng = np.random.default_rng(9)
    n = 33
    src, dst = _random_graph(rng, n)
    B = rng.standard_normal(n)
    X, _ = dense_solve(n, src, dst, D, B)
    g = oracle.Graph(n, src, dst)
    for name, (x, _) in _all_methods(g, B, D, 1e-13).items():
        assert np.abs(x - X).sum() <= 1e-13 / (1 - D) + 1e-13, name


def test_oracle_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.Graph(3, np.array([0, 0], np.int32), np.array([1, 1], np.int32))  # duplicate
    with pytest.raises(ValueError):
        oracle.Graph(3, np.array([0], np.int32), np.array([3], np.int32))  # range
    g = oracle.Graph(2, np.array([0], np.int32), np.array([1], np.int32))
    with pytest.raises(ValueError):
        oracle.diter(g, np.ones(2), 1.0)


def test_max_cycles_reports_noconv():
    g = oracle.Graph(3, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32))
    H, F, st = oracle.diter(g, np.ones(3), D, tol=1e-15, max_cycles=3)
    assert st.status == oracle.E_NOCONV and st.cycles == 3


def test_duplicate_check_on_unsorted_lists():
    src = np.array([0, 0, 0], np.int32)
    dst = np.array([2, 1, 2], np.int32)
    with pytest.raises(ValueError):
        oracle.Graph(3, src, dst)
    oracle.Graph(3, np.array([0, 0], np.int32), np.array([2, 1], np.int32))


@pytest.mark.parametrize("seed", range(4))
def test_power_iterates_against_matrix_powers(seed):
    """The unnormalized power (Jacobi) iteration starts at B and after m
    steps holds sum_{k<=m} P^k B (Section 2.5.1's update without the
    normalization); its residual is then |P^(m+1) B|_1. Checked against
    dense matrix powers, self-loops included."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(8, 30))
    src, dst = _random_graph(rng, n)
    g = oracle.Graph(n, src, dst)
    P = dense_p(n, src, dst, D)
    B = rng.random(n)
    for m in (0, 1, 5, 12):
        x, st = oracle.jacobi(g, B, D, tol=0.0, max_iter=m)
        assert st.status == oracle.E_NOCONV and st.cycles == m
        ref = sum(np.linalg.matrix_power(P, k) @ B for k in range(m + 1))
        assert np.allclose(x, ref, rtol=1e-13, atol=1e-15)
        r_ref = np.abs(np.linalg.matrix_power(P, m + 1) @ B).sum()
        assert abs(st.resid_l1 - r_ref) <= 1e-13 * max(r_ref, 1e-300) + 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_gauss_seidel_sweep_against_the_splitting(seed):
    """One ascending Gauss-Seidel sweep from x0 = B is the textbook
    splitting of A = I - P into its lower part L, diagonal D and upper part U:
    x1 = (D + L)^-1 (B - U x0). Checked with a dense triangular solve,
    self-loops (a diagonal of P) included."""
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(8, 30))
    src, dst = _random_graph(rng, n)
    g = oracle.Graph(n, src, dst)
    A = np.eye(n) - dense_p(n, src, dst, D)
    B = rng.random(n)
    lower = np.tril(A)
    upper = np.triu(A, 1)
    x = B.copy()
    for sweeps in (1, 2, 3):
        x = np.linalg.solve(lower, B - upper @ x)
        xs, st = oracle.gs(g, B, D, tol=0.0, max_sweeps=sweeps)
        assert st.status == oracle.E_NOCONV and st.cycles == sweeps
        assert np.allclose(xs, x, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_tiled_schedule_with_one_round_is_the_synchronous_one(seed):
    """One round per cycle: whatever the tiles, every cycle selects the same
    nodes, counts the same link operations and leaves the same F and H as
    the frontier-synchronous cycle (to the order of additions)."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(20, 60))
    src, dst = _random_graph(rng, n)
    g = oracle.Graph(n, src, dst)
    B = rng.random(n)
    for tile, reach in ((1, 0), (3, 1), (8, 4), (n, n)):
        Fs, Hs, Ft, Ht = B.copy(), np.zeros(n), B.copy(), np.zeros(n)
        es = et = 0.0
        for _ in range(12):
            cs, sels, es, ops_s, rs = oracle.di_cycle(g, Fs, Hs, D, oracle.SOP, oracle.SYNC, es)
            ct, selt, et, ops_t, rt = oracle.di_cycle(g, Ft, Ht, D, oracle.SOP, oracle.TILED, et,
                                                      tile=tile, reach=reach, rounds=1)
            assert (cs, ops_s) == (ct, ops_t) and np.array_equal(sels, selt)
            assert abs(rs - rt) <= 1e-15 * rs
            assert np.abs(Fs - Ft).sum() <= 1e-15 * B.sum()
            assert np.abs(Hs - Ht).sum() <= 1e-15 * Hs.sum()
            assert abs(es - et) <= 1e-15 * B.sum()


@pytest.mark.parametrize("tile", [1, 2, 3, 5, 12])
def test_tiled_schedule_on_a_path(tile):
    """A directed path 0 -> 1 -> ... -> 11 with all fluid on node 0: the
    fluid stays a single packet, of d^k b at node k. In the synchronous
    cycle it moves one node per cycle. In the tiled cycle with two rounds,
    the first round moves it one node and, if that step stayed inside the
    tile, the second round moves it once more; a step into the next tile
    waits for the next cycle. So the node it reaches after each cycle
    follows from the tile boundaries alone, and H holds d^k b for every node
    it has left. (Each node passes the DI-SOP threshold (r/L) out = r/11:
    the packet's value is r, and d r >= r/11.)"""
    n, b = 12, 0.15
    src = np.arange(n - 1, dtype=np.int32)
    dst = np.arange(1, n, dtype=np.int32)
    g = oracle.Graph(n, src, dst)
    F = np.zeros(n)
    F[0] = b
    H = np.zeros(n)
    e = 0.0
    pos = 0
    for cyc in range(12):
        # the packet's path this cycle: diffused at pos (absorbed if pos is
        # the dangling end, else sent to pos + 1); when pos + 1 lies in the
        # same tile, diffused there again in the second round
        cnt_x, ops_x, nxt, absorbed = 1, 0, pos, pos == n - 1
        if not absorbed:
            ops_x, nxt = 1, pos + 1
            if nxt // tile == pos // tile:
                cnt_x = 2
                if nxt == n - 1:
                    absorbed = True
                else:
                    ops_x, nxt = 2, nxt + 1
        cnt, _, e, ops, _ = oracle.di_cycle(g, F, H, D, oracle.SOP, oracle.TILED, e,
                                            tile=tile, reach=1, rounds=2)
        assert (cnt, ops) == (cnt_x, ops_x), (cyc, tile)
        if absorbed:
            assert F.sum() == 0.0 and e == pytest.approx(D ** (n - 1) * b, rel=1e-14)
            assert np.allclose(H, D ** np.arange(n) * b, rtol=1e-14, atol=0.0)
            break
        expect_F = np.zeros(n)
        expect_F[nxt] = D ** nxt * b
        assert np.allclose(F, expect_F, rtol=1e-14, atol=0.0), (cyc, tile)
        expect_H = np.array([D ** k * b if k < nxt else 0.0 for k in range(n)])
        assert np.allclose(H, expect_H, rtol=1e-14, atol=0.0), (cyc, tile)
        pos = nxt
    else:
        raise AssertionError("the packet was not absorbed")
