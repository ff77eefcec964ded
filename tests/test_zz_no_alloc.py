"""The allocation-free residual entry point against di_residual_dev, through
the C ABI on the GPU: the same R entry by entry and the same |R|_1 bit for
bit, on two calls in a row (the second on a smaller graph), and the size
limit rejected before any device work."""

import numpy as np
import pytest

from paper_1204_6255_amd import di, graphgen

pytestmark = pytest.mark.gpu

D = 0.85


def _dev_tensors(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    X = torch.tensor(rng.random(n) * 2.0 / n, dtype=torch.float64, device="cuda:0")
    B = torch.tensor(rng.random(n) * 0.3 / n, dtype=torch.float64, device="cuda:0")
    return X, B


@pytest.mark.parametrize("with_b", [True, False])
def test_noalloc_residual_matches_the_pooled_entry_point(with_b):
    import torch
    sizes = [(200_000, 1), (30_000, 2)]  # the second call is smaller
    for n, seed in sizes:
        print(f"noalloc residual: n={n} seed={seed} B={'given' if with_b else 'uniform'}",
              flush=True)
        src, dst = graphgen.web_graph(n, seed=seed)
        g = di.Graph(n, src, dst)
        X, B = _dev_tensors(n, seed)
        Bp = B if with_b else None
        R_ref = torch.empty(n, dtype=torch.float64, device="cuda:0")
        st, l1_ref = di.di_residual_dev(g.handle, Bp, D, X, R_ref)
        assert st == di.DI_OK, di.di_last_error()
        R = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        st, l1 = di.di_residual_dev_noalloc(g.handle, Bp, D, X, R)
        assert st == di.DI_OK, di.di_last_error()
        torch.cuda.synchronize()
        assert l1 == l1_ref  # the same pass and the same fold order
        assert torch.equal(R, R_ref)
        # R kept in the scratch array: only the norm comes back
        st, l1b = di.di_residual_dev_noalloc(g.handle, Bp, D, X, None)
        assert st == di.DI_OK, di.di_last_error()
        assert l1b == l1_ref
        g.close()


def test_noalloc_residual_with_a_heavy_row_and_self_loops():
    import torch
    n = 40_000
    src, dst = graphgen.web_graph(n, seed=5)
    # a hub with 30,000 in-links (split into segments) and self-loops
    extra_src = np.arange(1, 30_001, dtype=np.int32)
    extra_dst = np.zeros(30_000, dtype=np.int32)
    loops = np.arange(0, n, 97, dtype=np.int32)
    s = np.concatenate([src, extra_src, loops])
    t = np.concatenate([dst, extra_dst, loops])
    key = np.unique(s.astype(np.int64) * n + t)
    s, t = (key // n).astype(np.int32), (key % n).astype(np.int32)
    print(f"noalloc residual: hub graph n={n} links={s.size}", flush=True)
    g = di.Graph(n, s, t)
    X, B = _dev_tensors(n, 9)
    R_ref = torch.empty(n, dtype=torch.float64, device="cuda:0")
    st, l1_ref = di.di_residual_dev(g.handle, B, D, X, R_ref)
    assert st == di.DI_OK
    R = torch.empty(n, dtype=torch.float64, device="cuda:0")
    st, l1 = di.di_residual_dev_noalloc(g.handle, B, D, X, R)
    assert st == di.DI_OK, di.di_last_error()
    torch.cuda.synchronize()
    assert l1 == l1_ref and torch.equal(R, R_ref)
    g.close()


def test_noalloc_residual_rejects_a_graph_beyond_the_scratch_size():
    import torch
    n = 20_000_000  # 8n doubles of y alone exceed 128 MiB
    print(f"noalloc residual: size limit n={n}", flush=True)
    g = di.Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    X = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    R = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    st, _ = di.di_residual_dev_noalloc(g.handle, None, D, X, R)
    assert st == di.DI_E_INVAL
    assert "scratch" in di.di_last_error()
    g.close()
