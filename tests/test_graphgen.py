"""The seeded input generator and the Table-1 statistics."""

import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1204_6255_amd import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_deterministic_per_seed_and_seed_sensitive():
    a = graphgen.web_graph(5000, seed=3)
    b = graphgen.web_graph(5000, seed=3)
    c = graphgen.web_graph(5000, seed=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0].size != c[0].size or not np.array_equal(a[1], c[1])


def test_independent_of_thread_count():
    code = ("import sys; sys.path.insert(0, %r); import hashlib; "
            "from paper_1204_6255_amd import graphgen; "
            "s, d = graphgen.web_graph(200000, seed=1); "
            "print(hashlib.sha256(s.tobytes() + d.tobytes()).hexdigest())") % ROOT
    outs = []
    for threads in ("1", "5"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout.strip())
    assert outs[0] == outs[1]


@pytest.mark.parametrize("alpha", [graphgen.ALPHA_L_MATCHED, graphgen.ALPHA_LITERAL])
def test_sorted_unique_no_self_loops_in_range(alpha):
    n = 20000
    src, dst = graphgen.web_graph(n, seed=0, alpha=alpha)
    assert src.dtype == np.int32 and dst.dtype == np.int32
    assert src.min() >= 0 and src.max() < n and dst.min() >= 0 and dst.max() < n
    key = src.astype(np.int64) * n + dst
    assert np.all(np.diff(key) > 0)  # strictly increasing: sorted and unique
    assert not np.any(src == dst)


def test_realized_statistics_at_10k():
    n = 10000
    src, dst = graphgen.web_graph(n, seed=0)
    st = graphgen.graph_stats(n, src, dst)
    row = st.table1_row()
    assert 7.0 < row["L/N"] < 8.2  # L-matched exponent: L close to 76k
    assert 0.13 < row["D/N"] < 0.17
    assert st.O == 0 and st.max_out <= 500
    src2, dst2 = graphgen.web_graph(n, seed=0, alpha=graphgen.ALPHA_LITERAL)
    assert 2.4 < graphgen.graph_stats(n, src2, dst2).L / n < 3.2


def test_local_link_fraction_and_radius():
    n = 100000
    src, dst = graphgen.web_graph(n, seed=2)
    off = dst.astype(np.int64) - src
    local = np.abs(off) <= 500
    # 70% local draws plus the Zipf draws that land nearby by chance
    assert 0.66 < local.mean() < 0.75


def _brute_stats(n, src, dst):
    out = np.bincount(src, minlength=n)
    ind = np.bincount(dst, minlength=n)
    # E by its definition: grow the set of nodes whose in-links all come from
    # the set, until nothing changes
    E = np.zeros(n, bool)
    changed = True
    while changed:
        changed = False
        for i in range(n):
            if not E[i] and all(E[j] for j in src[dst == i]):
                E[i] = True
                changed = True
    return dict(L=len(src), D=int(np.sum(out == 0)), zero_in=int(np.sum(ind == 0)),
                E=int(E.sum()), O=int(np.sum(src == dst)),
                max_in=int(ind.max(initial=0)), max_out=int(out.max(initial=0)))


@pytest.mark.parametrize("seed", range(6))
def test_table1_stats_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 25))
    mask = rng.random((n, n)) < rng.uniform(0.02, 0.3)
    src, dst = (a.astype(np.int32) for a in np.nonzero(mask))
    st = graphgen.graph_stats(n, src, dst)
    ref = _brute_stats(n, src, dst)
    for k, v in ref.items():
        assert getattr(st, k) == v, (k, getattr(st, k), v)


def test_ppr_inputs():
    sets = graphgen.ppr_seed_sets(1000, 8)
    assert len(sets) == 8
    for s in sets:
        assert 1 <= s.size <= 100 and np.unique(s).size == s.size
    b = graphgen.ppr_rhs(1000, sets[0], 0.85)
    assert abs(b.sum() - 0.15) < 1e-15 and np.count_nonzero(b) == sets[0].size
    assert all(np.array_equal(x, y) for x, y in zip(sets, graphgen.ppr_seed_sets(1000, 8)))


def test_small_and_degenerate_sizes():
    for n in (0, 1, 2, 3):
        src, dst = graphgen.web_graph(n, seed=0)
        assert src.size == dst.size
        if n < 2:
            assert src.size == 0
        else:
            assert np.all(src != dst) and np.all(dst < n)
    with pytest.raises(ValueError):
        graphgen.web_graph(-1)


def test_transpose_and_prefix_subgraph():
    n = 3000
    src, dst = graphgen.web_graph(n, seed=4)
    ts, td = graphgen.transpose(src, dst)
    # sorted by (origin, destination), the same link set reversed
    key = ts.astype(np.int64) * n + td
    assert np.all(np.diff(key) > 0)
    assert set(zip(ts.tolist(), td.tolist())) == set(zip(dst.tolist(), src.tolist()))
    st = graphgen.graph_stats(n, src, dst)
    tt = graphgen.graph_stats(n, ts, td)
    assert tt.L == st.L and tt.max_in == st.max_out and tt.max_out == st.max_in
    # transposing twice gives the original list back
    bs, bd = graphgen.transpose(ts, td)
    assert np.array_equal(bs, src) and np.array_equal(bd, dst)
    m = 1000
    ps, pd = graphgen.prefix_subgraph(m, src, dst)
    assert np.all(ps < m) and np.all(pd < m)
    expect = [(a, b) for a, b in zip(src.tolist(), dst.tolist()) if a < m and b < m]
    assert list(zip(ps.tolist(), pd.tolist())) == expect


def test_forward_links_give_a_dag():
    """p_forward = 1 with local links only: every link points forward, so
    every node converges in finitely many steps (E = N); p_forward = 0
    leaves the generator's output unchanged."""
    n = 5000
    s, d = graphgen.web_graph(n, seed=2, alpha=graphgen.ALPHA_LITERAL, p_dangling=0.48,
                              p_local=1.0, p_forward=1.0)
    assert np.all(d > s)
    st = graphgen.graph_stats(n, s, d)
    assert st.E == n and st.zero_in >= 1
    a = graphgen.web_graph(n, seed=2)
    b = graphgen.web_graph(n, seed=2, p_forward=0.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_peel_against_the_definition():
    """The peel helper's E class equals the definition's fixed point."""
    from _peel import e_depth
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        n = int(rng.integers(1, 25))
        mask = rng.random((n, n)) < rng.uniform(0.02, 0.3)
        src, dst = (a.astype(np.int32) for a in np.nonzero(mask))
        assert int((e_depth(n, src, dst) >= 0).sum()) == _brute_stats(n, src, dst)["E"]
    # a chain 0 -> 1 -> 2 with 3 <-> 4 -> 2: node 2 has a cycle upstream
    depth = e_depth(5, [0, 1, 3, 4, 4], [1, 2, 4, 3, 2])
    assert depth.tolist() == [0, 1, -1, -1, -1]


def test_high_e_graph_matches_table9():
    """Section 2.8's graph at N = 9664: L/N 1.67, D/N 0.48, E/N 0.91, no
    loops, max_in near 199, max_out at most 164."""
    from _peel import e_depth
    n = 9664
    src, dst = graphgen.high_e_graph(n, seed=0)
    key = src.astype(np.int64) * n + dst
    assert np.all(np.diff(key) > 0) and np.all(src != dst)
    assert src.min() >= 0 and dst.max() < n
    st = graphgen.graph_stats(n, src, dst)
    assert st.L == round(1.67 * n)
    assert st.D == round(0.48 * n) and st.O == 0
    assert st.E == n - round(0.09 * n)
    assert int((e_depth(n, src, dst) >= 0).sum()) == st.E
    assert st.max_out <= 164 and 100 <= st.max_in <= 400
    a = graphgen.high_e_graph(n, seed=0)
    b = graphgen.high_e_graph(n, seed=1)
    assert np.array_equal(a[0], src) and np.array_equal(a[1], dst)
    assert not (a[0].size == b[0].size and np.array_equal(a[1], b[1]))
    # small sizes keep the construction (a ring of at least 2 nodes)
    for m in (4, 10, 50):
        s, t = graphgen.high_e_graph(m, seed=0)
        sm = graphgen.graph_stats(m, s, t)
        assert sm.O == 0 and sm.E == m - max(2, round(0.09 * m))
    with pytest.raises(ValueError):
        graphgen.high_e_graph(3)
