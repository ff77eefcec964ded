"""Benchmark: time to an L1 residual of 1e-9 for DI-SOP PageRank on one GPU.

Workload: the synthetic web graph with N = 1,000,000 nodes (seed 0,
out-degree power law with exponent 1.68 on [1, 500], 15% dangling nodes,
70% of links within +-500 ids, the rest Zipf(1) over a random permutation),
d = 0.85, B = (1-d)/N, FP64 fluid, stop at sum |F| <= 1e-9. Inputs are
resident in HBM before the timed region; one step is one full solve.

Prints one JSON line. `value` is the mean wall time per solve over the
timed steps. The roofline object is for the kernel that moves the fluid
(the window push, which also selects, unless the graph's tuning picked the
CSC pull): the method's bytes per launch over its mean launch time,
measured with HIP events around each launch in a second pass of the same
steps (events add stream packets, so they stay out of `value`). The
cpu_baseline object times the CPU oracle (sequential DI-SOP, one thread)
on the same graph.

The same line also reports, on the same graph unless stated:
  fp32_refine   the same solve with FP32 fluid and FP64 residual passes;
  methods, literal_alpha_1m, config_10k, transposed_1m, dataset2_like,
  prefix_sweep  the other methods and kernels, the literal exponent, N = 10k,
                the transposed graph, the high-E stand-in and the prefix
                subgraphs (each with the tuner's choice for its graph);
  batched_ppr   personalized PageRank batches (k = 8, 64, 256 seed sets of
                1..100 nodes, tol 1e-9 each, FP32 + FP64 refinement, one
                batch per call): solves/s, against single FP64 solves of the
                same right-hand sides;
  serving       32 graphs with N log-uniform in [1e4, 5e6] (seeds 1..32);
                requests pick a graph uniformly, a seed set of 1..100 nodes
                and tol 1e-6 or 1e-9 (50/50); closed loop with 1024
                requests in flight gives the saturated rate mu, then Poisson
                arrivals at 0.5 mu and 0.8 mu: solves/s, p50 / p99 latency
                (submission to completion), admission stalls.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N]
                       [--no-extras] [--serve-seconds S]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
CSRC = os.path.join(ROOT, "paper_1204_6255_amd", "csrc")
# per move kernel: its committed counter summary and the source it was taken on
TRAFFIC = {
    "window": (os.path.join(ROOT, "profiles", "k_wcycle_f64_n1m_traffic.txt"),
               os.path.join(CSRC, "di_window.hip")),
    "pull": (os.path.join(ROOT, "profiles", "k_pull_f64_n1m_traffic.txt"),
             os.path.join(CSRC, "di_kernels.hip")),
}


def parse_args():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=1_000_000)
    p.add_argument("--alpha", type=float, default=1.68)
    p.add_argument("--kmax", type=int, default=500, help="largest out-degree of the generator")
    p.add_argument("--precision", choices=["fp64", "fp32", "fp32r"], default="fp64",
                   help="fluid precision (fp32r: FP32 with FP64 residual passes)")
    p.add_argument("--tol", type=float, default=1e-9)
    p.add_argument("--kernel", choices=["auto", "pull", "push", "window"], default="auto")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="budget of the CPU-oracle sample (0 disables it)")
    p.add_argument("--no-extras", action="store_true",
                   help="headline solve only (no FP32, method, high-E, batched or serving sections)")
    p.add_argument("--only", choices=["fp32_refine", "methods", "literal_alpha_1m", "config_10k",
                                      "transposed_1m",
                                      "dataset2_like", "prefix_sweep", "batched_ppr", "serving"],
                   default=None,
                   help="run this one section after the headline solve (for profiling)")
    p.add_argument("--serve-seconds", type=float, default=6.0,
                   help="length of each serving phase")
    p.add_argument("--serve-kmax", type=int, default=16)
    p.add_argument("--window-cfg", default=None, metavar="TILE,HUBS,GRID[,ROUNDS]",
                   help="pin the window configuration of the headline graph instead of tuning it "
                        "(for profiler runs, whose timing would steer the tuner)")
    p.add_argument("--calibration-copy", action="store_true",
                   help="after the timed region, fill 1 GiB and then sum it (a write-only and a "
                        "read-only kernel of known size, for scaling memory counters)")
    return p.parse_args()


def kernel_source_hash(path) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(kind):
    """Measured HBM bytes per launch of the move kernel (`window` or `pull`)
    from the committed counter summary, or None when it is missing or was
    taken on other kernel source."""
    path, source = TRAFFIC[kind]
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("kernel_source_sha256_16") != kernel_source_hash(source):
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_methods(oracle, og, B, d, tol):
    """The oracle's five methods on one graph: resid mode to tol (time,
    iterations, nb_iter), and nb_iter in the paper's mode (target 1/N)."""
    n = og.n
    out = {}
    for name, variant in (("DI-SOP", oracle.SOP), ("DI-CYC", oracle.CYC)):
        _, _, st = oracle.diter(og, B, d, variant, oracle.SEQUENTIAL, tol=tol)
        _, _, sp = oracle.diter(og, B, d, variant, oracle.SEQUENTIAL, stop=oracle.STOP_PAPER,
                                tol=1.0 / n)
        out[name] = {"s": st.seconds, "cycles": int(st.cycles), "nb_iter": st.nb_iter,
                     "paper_mode_nb_iter": sp.nb_iter}
    _, st = oracle.jacobi(og, B, d, tol=tol)
    _, sp = oracle.pi(og, d)
    _, sq = oracle.pi(og, d, by_columns=True)
    out["PI (power/Jacobi iteration)"] = {"s": st.seconds, "iterations": int(st.cycles),
                                          "nb_iter": st.nb_iter,
                                          "paper_mode_nb_iter": sp.nb_iter,
                                          "paper_mode_nb_iter_PI'": sq.nb_iter}
    _, st = oracle.gs(og, B, d, stop=oracle.STOP_RESID, tol=tol)
    _, sp = oracle.gs(og, B, d, stop=oracle.STOP_PAPER, tol=1.0 / n)
    out["GS (sequential sweep)"] = {"s": st.seconds, "sweeps": int(st.cycles),
                                    "nb_iter": st.nb_iter, "paper_mode_nb_iter": sp.nb_iter}
    return out


def cpu_baseline(n, d, tol, budget_s, alpha, kmax, solutions=None, with_baselines=True):
    """The oracle on the host: repeated DI-SOP solves of the benchmark graph
    (the baseline value), its other methods once each, the N = 10k
    configuration, and the L1 error of every GPU solution collected by the
    other sections against an oracle solve to 1e-13."""
    import numpy as np
    import oracle
    from paper_1204_6255_amd import graphgen

    graphs = {}

    def graph(key):
        if key not in graphs:
            m, a = {"1m": (n, alpha), "1m_a2.1": (n, graphgen.ALPHA_LITERAL)}[key]
            s_, t_ = graphgen.web_graph(m, seed=0, alpha=a, kmax=kmax)
            graphs[key] = oracle.Graph(m, s_, t_)
        return graphs[key]

    og = graph("1m")
    B = graphgen.uniform_rhs(n, d)
    times = []
    t_start = time.perf_counter()
    while True:
        _, _, st = oracle.diter(og, B, d, oracle.SOP, oracle.SEQUENTIAL, tol=tol)
        times.append(st.seconds)
        if time.perf_counter() - t_start >= budget_s or len(times) >= 50:
            break
    out = {
        "value": float(np.mean(times)), "unit": "s", "cores": 1, "kind": "oracle",
        "sample": f"{len(times)} full solves of the same N={n} graph to sum|F| <= {tol:g} "
                  f"(sequential DI-SOP, one thread, FP64)",
        "host_cpu": host_cpu(), "host_nproc": os.cpu_count(),
    }
    if not with_baselines:
        return out
    out["oracle_baselines"] = oracle_methods(oracle, og, B, d, tol)
    # the N = 10k configuration at both readings of the out-degree exponent
    small = {}
    for a in (graphgen.ALPHA_L_MATCHED, graphgen.ALPHA_LITERAL):
        s_, t_ = graphgen.web_graph(10_000, seed=0, alpha=a, kmax=kmax)
        small[f"alpha={a}"] = oracle_methods(oracle, oracle.Graph(10_000, s_, t_),
                                             graphgen.uniform_rhs(10_000, d), d, tol)
    out["oracle_n10k"] = small
    # the oracle's side of the prefix sweep (Tables 2-3): sequential DI-SOP
    # nb_iter per N, both stop modes
    s_full, t_full = graphgen.web_graph(n, seed=0, alpha=alpha, kmax=kmax)
    sweep = []
    for m in PREFIX_SIZES:
        if m > n:
            break
        s_, t_ = graphgen.prefix_subgraph(m, s_full, t_full)
        og_ = og if m == n else oracle.Graph(m, s_, t_)
        Bm = graphgen.uniform_rhs(m, d)
        _, _, st = oracle.diter(og_, Bm, d, oracle.SOP, oracle.SEQUENTIAL, tol=tol)
        _, _, sp = oracle.diter(og_, Bm, d, oracle.SOP, oracle.SEQUENTIAL, stop=oracle.STOP_PAPER,
                                tol=1.0 / m)
        sweep.append({"N": m, "resid_s": st.seconds, "resid_nb_iter": st.nb_iter,
                      "resid_cycles": int(st.cycles), "paper_nb_iter": sp.nb_iter,
                      "paper_cycles": int(sp.cycles)})
    out["oracle_prefix_sweep"] = sweep
    del s_full, t_full
    # error of every collected GPU solution against the oracle's
    if solutions:
        refs, errs = {}, {}
        for name, (gkey, bkey, X) in solutions.items():
            if (gkey, bkey) not in refs:
                og_ = graph(gkey)
                if bkey == "uniform":
                    Bk = graphgen.uniform_rhs(og_.n, d)
                else:
                    k, j = bkey
                    Bk = graphgen.ppr_rhs(og_.n, graphgen.ppr_seed_sets(og_.n, k)[j], d)
                refs[(gkey, bkey)], _, _ = oracle.diter(og_, Bk, d, oracle.SOP,
                                                        oracle.SEQUENTIAL, tol=1e-13)
            errs[name] = float(np.abs(X - refs[(gkey, bkey)]).sum())
        out["error_vs_oracle_l1"] = errs
        out["error_vs_oracle_note"] = ("L1 distance to the oracle's DI-SOP solve to 1e-13 "
                                       "(itself within 1e-13/(1-d) of the exact X); a solve to "
                                       "tol is within tol/(1-d)")
    return out


def time_solves(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [fn() for _ in range(reps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out[-1]


def fp32_refine_section(di, g, X, d, tol, solutions):
    o = di.di_opts_default()
    o.precision = di.DI_FP32_REFINE

    def solve():
        status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        return st

    sec, st = time_solves(solve, 10)
    solutions["DI-SOP pull fp32+refine"] = ("1m", "uniform", X.cpu().numpy())
    return {"s_per_solve": sec, "cycles": int(st.cycles), "refinements": int(st.refinements),
            "resid_l1": float(st.resid_l1)}


def methods_section(di, g, X, d, tol, solutions):
    """The paper's method comparison on the GPU, same graph and tolerance:
    DI-SOP, DI-CYC and PI, each moving fluid by the pull (rows gathered, as
    PI), by the atomic push (columns scattered, as PI') and by the window
    push (one launch per cycle, only the moved links read). PI diffuses
    every node every cycle, so its history after m + 1 cycles is the power
    iteration's iterate after m steps, at the power iteration's cost."""
    rows = []
    for name, method in (("DI-SOP", di.DI_SOP), ("DI-CYC", di.DI_CYC), ("PI", di.DI_PI)):
        for kname, kernel in (("pull", di.DI_KERNEL_PULL), ("push", di.DI_KERNEL_PUSH),
                              ("window", di.DI_KERNEL_WINDOW)):
            o = di.di_opts_default()
            o.method = method
            o.kernel = kernel

            def solve():
                status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
                if status != di.DI_OK:
                    raise RuntimeError(di.di_last_error())
                return st

            sec, st = time_solves(solve, 5)
            rows.append({"method": name, "kernel": kname, "ms_per_solve": sec * 1e3,
                         "cycles": int(st.cycles), "nb_iter": float(st.nb_iter),
                         "resid_l1": float(st.resid_l1)})
            solutions[f"{name} {kname} fp64"] = ("1m", "uniform", X.cpu().numpy())
    # PI in FP32 with FP64 residual passes
    o = di.di_opts_default()
    o.method = di.DI_PI
    o.precision = di.DI_FP32_REFINE

    def pi32():
        status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        return st

    sec, st = time_solves(pi32, 5)
    rows.append({"method": "PI", "kernel": "pull", "precision": "fp32+fp64 refinement",
                 "ms_per_solve": sec * 1e3, "cycles": int(st.cycles), "nb_iter": float(st.nb_iter),
                 "refinements": int(st.refinements), "resid_l1": float(st.resid_l1)})
    solutions["PI pull fp32+refine"] = ("1m", "uniform", X.cpu().numpy())
    # the Gauss-Seidel baseline as an asynchronous in-place relaxation
    o = di.di_opts_default()
    o.method = di.DI_GS_ASYNC

    def gs():
        status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        return st

    sec, st = time_solves(gs, 5)
    rows.append({"method": "GS-async (GPU variant)", "kernel": "pull", "ms_per_solve": sec * 1e3,
                 "cycles": int(st.cycles), "nb_iter": float(st.nb_iter),
                 "resid_l1": float(st.resid_l1)})
    solutions["GS-async pull fp64"] = ("1m", "uniform", X.cpu().numpy())
    return rows


def literal_alpha_section(di, graphgen, n, d, tol, kmax, solutions):
    """The N = 1M graph at the literal out-degree exponent 2.1 (about 2.8
    links per node): DI-SOP in FP64 and FP32 with FP64 refinement."""
    import torch
    src, dst = graphgen.web_graph(n, seed=0, alpha=graphgen.ALPHA_LITERAL, kmax=kmax)
    st_g = graphgen.graph_stats(n, src, dst)
    g = di.Graph(n, src, dst)
    del src, dst
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    out = {"alpha": graphgen.ALPHA_LITERAL, "links": int(st_g.L), "dangling": int(st_g.D),
           "zero_in": int(st_g.zero_in), "rows": []}
    for pname, prec in (("fp64", di.DI_FP64), ("fp32+refine", di.DI_FP32_REFINE)):
        o = di.di_opts_default()
        o.precision = prec

        def solve():
            status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
            if status != di.DI_OK:
                raise RuntimeError(di.di_last_error())
            return st

        sec, st = time_solves(solve, 10)
        out["rows"].append({"precision": pname, "ms_per_solve": sec * 1e3, "cycles": int(st.cycles),
                            "nb_iter": float(st.nb_iter), "resid_l1": float(st.resid_l1),
                            "gedges_per_s": st.edges_pushed / sec / 1e9})
        solutions[f"alpha 2.1 DI-SOP {pname}"] = ("1m_a2.1", "uniform", X.cpu().numpy())
    out["tuning"] = di.di_graph_tuning(g.handle)
    g.close()
    return out


def small_graph_section(di, graphgen, d, tol):
    """The N = 10k configuration (launch-latency bound), both exponents."""
    import torch
    out = []
    for a in (graphgen.ALPHA_L_MATCHED, graphgen.ALPHA_LITERAL):
        src, dst = graphgen.web_graph(10_000, seed=0, alpha=a)
        g = di.Graph(10_000, src, dst)
        X = torch.empty(10_000, dtype=torch.float64, device="cuda")
        o = di.di_opts_default()

        def solve():
            status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
            if status != di.DI_OK:
                raise RuntimeError(di.di_last_error())
            return st

        sec, st = time_solves(solve, 20)
        out.append({"alpha": a, "links": int(len(src)), "ms_per_solve": sec * 1e3,
                    "cycles": int(st.cycles), "nb_iter": float(st.nb_iter),
                    "tuning": di.di_graph_tuning(g.handle)})
        g.close()
    return out


def transposed_section(di, graphgen, n, d, tol, alpha, kmax):
    """Section 2.7's workload: the benchmark graph with every link
    reversed (Pt), FP64 DI-SOP to the same residual, and what the tuner
    picked for it (its hub rows are the original's hubs of out-links)."""
    import torch
    src, dst = graphgen.web_graph(n, seed=0, alpha=alpha, kmax=kmax)
    s, t = graphgen.transpose(src, dst)
    del src, dst
    g = di.Graph(n, s, t)
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    o = di.di_opts_default()

    def solve():
        status, st = di.di_solve_dev(g.handle, None, d, tol, o, X)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        return st

    sec, st = time_solves(solve, 10)
    out = {"graph": f"transpose of the N={n} benchmark graph", "ms_per_solve": sec * 1e3,
           "cycles": int(st.cycles), "nb_iter": float(st.nb_iter), "resid_l1": float(st.resid_l1),
           "tuning": di.di_graph_tuning(g.handle)}
    g.close()
    return out


def high_e_section(di, graphgen, d):
    """Section 2.8's graph (Table 9) by its synthetic stand-in, on P and its
    transpose: DI-SOP and DI-CYC to the paper's target error 1/N, where
    most nodes converge exactly in finitely many steps."""
    import torch
    n = 9664
    out = {"graph": f"high-E stand-in N={n} seed 0 (L/N 1.67, D/N 0.48, E/N 0.91)",
           "stop": "paper, target 1/N", "rows": []}
    base = graphgen.high_e_graph(n, seed=0)
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    for mat, (src, dst) in (("P", base), ("Pt", graphgen.transpose(*base))):
        g = di.Graph(n, src, dst)
        for name, method in (("DI-SOP", di.DI_SOP), ("DI-CYC", di.DI_CYC)):
            o = di.di_opts_default()
            o.method = method
            o.stop = di.DI_STOP_PAPER

            def solve():
                status, st = di.di_solve_dev(g.handle, None, d, 1.0 / n, o, X)
                if status != di.DI_OK:
                    raise RuntimeError(di.di_last_error())
                return st

            sec, st = time_solves(solve, 20)
            out["rows"].append({"matrix": mat, "method": name, "us_per_solve": sec * 1e6,
                                "cycles": int(st.cycles), "nb_iter": float(st.nb_iter)})
        out.setdefault("tuning", {})[mat] = di.di_graph_tuning(g.handle)
        g.close()
    return out


PREFIX_SIZES = (1_000, 10_000, 100_000, 1_000_000)


def prefix_sweep_section(di, graphgen, n, d, tol, alpha, kmax):
    """Section 2.6's scaling method on the synthetic stand-in: the subgraphs
    induced on the first N ids of the benchmark graph, N = 10^3 .. 10^6,
    with the statistics of Table 1, and DI-SOP's GPU time, cycles and cost
    (nb_iter) per N in both stop modes (the GPU's side of Tables 2-3; the
    oracle's nb_iter for the same subgraphs is in cpu_baseline)."""
    import torch
    src, dst = graphgen.web_graph(n, seed=0, alpha=alpha, kmax=kmax)
    rows = []
    for m in PREFIX_SIZES:
        if m > n:
            break
        s, t = graphgen.prefix_subgraph(m, src, dst)
        row = graphgen.graph_stats(m, s, t).table1_row()
        g = di.Graph(m, s, t)
        X = torch.empty(m, dtype=torch.float64, device="cuda")
        for mode, stop, tl in (("resid", di.DI_STOP_RESID, tol), ("paper", di.DI_STOP_PAPER, 1.0 / m)):
            o = di.di_opts_default()
            o.stop = stop

            def solve():
                status, st = di.di_solve_dev(g.handle, None, d, tl, o, X)
                if status != di.DI_OK:
                    raise RuntimeError(di.di_last_error())
                return st

            sec, st = time_solves(solve, 10 if m < n else 5)
            row[f"gpu_{mode}"] = {"ms_per_solve": sec * 1e3, "cycles": int(st.cycles),
                                  "nb_iter": float(st.nb_iter),
                                  "resid_l1": float(st.resid_l1),
                                  "gedges_per_s": st.edges_pushed / sec / 1e9}
        row["tuning"] = di.di_graph_tuning(g.handle)
        rows.append(row)
        g.close()
    return {"graph": f"prefixes of the N={n} benchmark graph (ids < N, induced)",
            "tol_resid": tol, "paper_target": "1/N", "rows": rows}


def batched_section(di, graphgen, g, n, d, tol, solutions):
    import numpy as np
    import torch
    out = {"precision": "fp32+fp64 refinement", "tol": tol, "seed_sets": "1..100 nodes, seed 1000+j"}
    # single FP64 solves of the first right-hand side, for comparison
    B0 = torch.from_numpy(graphgen.ppr_rhs(n, graphgen.ppr_seed_sets(n, 1)[0], d)).cuda()
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    o64 = di.di_opts_default()

    def single():
        status, st = di.di_solve_dev(g.handle, B0, d, tol, o64, X)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        return st

    sec1, _ = time_solves(single, 5)
    out["single_fp64_solves_per_s"] = 1.0 / sec1
    runs = []
    for k in (8, 64, 256):
        B = np.stack([graphgen.ppr_rhs(n, s, d) for s in graphgen.ppr_seed_sets(n, k)])
        Bd = torch.from_numpy(B).cuda()
        Xd = torch.empty((k, n), dtype=torch.float64, device="cuda")
        o = di.di_opts_default()
        o.precision = di.DI_FP32_REFINE

        def batch():
            status, st = di.di_solve_batch_dev(g.handle, k, Bd, d, tol, o, Xd)
            if status != di.DI_OK:
                raise RuntimeError(di.di_last_error())
            return st

        sec, st = time_solves(batch, 2)
        Xh = Xd[:2].cpu().numpy()
        for j in range(2):
            solutions[f"batched k={k} column {j}"] = ("1m", (k, j), Xh[j].copy())
        runs.append({"k": k, "s_per_batch": sec, "solves_per_s": k / sec,
                     "vs_single_fp64": (k / sec) * sec1,
                     "max_cycles": max(x.cycles for x in st),
                     "max_resid_l1": max(x.resid_l1 for x in st)})
        del Bd, Xd
        torch.cuda.empty_cache()
    out["runs"] = runs
    return out


def serving_section(di, graphgen, d, seconds, kmax):
    import numpy as np
    ng = 32
    Ns = [int(round(np.exp(np.random.default_rng(gid).uniform(np.log(1e4), np.log(5e6)))))
          for gid in range(1, ng + 1)]
    graphs = []
    for gid, n in enumerate(Ns, 1):
        s, t = graphgen.web_graph(n, seed=gid)
        graphs.append(di.Graph(n, s, t))
    status, srv = di.di_serve_create(200 << 30, kmax)
    if status != di.DI_OK:
        raise RuntimeError(di.di_last_error())
    t0 = time.perf_counter()
    for gid, G in enumerate(graphs):
        if di.di_serve_add_graph(srv, G.handle, gid) != di.DI_OK:
            raise RuntimeError(di.di_last_error())
    add_seconds = time.perf_counter() - t0
    bufs = [np.empty(n) for n in Ns]

    def request(i):
        r = np.random.default_rng(1_000_000 + i)
        gid = int(r.integers(0, ng))
        size = int(r.integers(1, 101))
        seeds = r.choice(Ns[gid], size=size, replace=False).astype(np.int32)
        return gid, seeds, (1e-6 if r.random() < 0.5 else 1e-9)

    counter = [0]

    def submit(inflight):
        gid, seeds, tol = request(counter[0])
        counter[0] += 1
        st, tk = di.di_serve_submit(srv, gid, seeds, d, tol)
        if st != di.DI_OK:
            raise RuntimeError(di.di_last_error())
        inflight[tk] = gid

    def reap(inflight, lat, parts=None):
        for tk in list(inflight):
            st, sts = di.di_serve_poll(srv, tk, bufs[inflight[tk]])
            if st != di.DI_PENDING:
                if st != di.DI_OK:
                    raise RuntimeError(di.di_last_error())
                del inflight[tk]
                lat.append(sts.seconds)
                if parts is not None:
                    parts.append((sts.queue_seconds, sts.run_seconds, sts.readout_seconds,
                                  sts.refinements == 0))

    def breakdown(parts):
        """The latency split of the requests: waiting for a slot or column,
        running, reading out (p50 and mean, ms), and the share that ran on
        the single right-hand side path."""
        a = np.array([p[:3] for p in parts])
        out = {}
        for k, name in enumerate(("queue", "run", "readout")):
            out[name + "_p50_ms"] = 1e3 * float(np.percentile(a[:, k], 50))
            out[name + "_mean_ms"] = 1e3 * float(a[:, k].mean())
        out["single_path_share"] = float(np.mean([p[3] for p in parts]))
        return out

    def drain(inflight):
        while inflight:
            reap(inflight, [])
            time.sleep(0.001)

    # closed loop: 1024 requests in flight
    inflight, lat, parts = {}, [], []
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        while len(inflight) < 1024:
            submit(inflight)
        reap(inflight, lat, parts)
        time.sleep(0.0005)
    el = time.perf_counter() - t0
    mu = len(lat) / el
    closed = {"in_flight": 1024, "solves_per_s": mu, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
              "p99_ms": 1e3 * float(np.percentile(lat, 99)), "requests": len(lat),
              "breakdown": breakdown(parts)}
    drain(inflight)
    poisson = []
    for frac in (0.5, 0.8):
        lam = frac * mu
        nreq = int(min(10000, lam * seconds))
        arr = np.cumsum(np.random.default_rng(int(frac * 10)).exponential(1.0 / lam, nreq))
        inflight, lat, parts = {}, [], []
        t0 = time.perf_counter()
        q = 0
        while q < nreq or inflight:
            now = time.perf_counter() - t0
            while q < nreq and arr[q] <= now:
                submit(inflight)
                q += 1
            reap(inflight, lat, parts)
            time.sleep(0.0002)
        el = time.perf_counter() - t0
        poisson.append({"lambda_per_s": lam, "requests": nreq, "solves_per_s": nreq / el,
                        "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                        "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                        "breakdown": breakdown(parts)})
    # idle: one request at a time (each runs alone on its graph); the same
    # requests in every run, whatever the earlier phases submitted
    counter[0] = 20_000_000
    lat, parts = [], []
    for i in range(64):
        inflight = {}
        submit(inflight)
        while inflight:
            reap(inflight, lat, parts)
            time.sleep(0.0001)
    idle = {"requests": len(lat), "p50_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat, 99)), "breakdown": breakdown(parts)}
    _, info = di.di_serve_info(srv)
    di.di_serve_destroy(srv)
    for G in graphs:
        G.close()
    return {"graphs": ng, "total_nodes": int(sum(Ns)), "k_max": kmax,
            "precision": "fp32+fp64 refinement in column sets; fp64 single path in solo slots",
            "solo_requests": int(info.solo_requests),
            "add_graphs_s": add_seconds,
            "closed_loop": closed, "poisson": poisson, "idle_one_at_a_time": idle,
            "admission_stalls": int(info.admission_stalls),
            "hbm_bytes_in_use": int(info.bytes_in_use)}


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "design is described in the design notes and is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1204_6255_amd import di, graphgen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, d, tol = args.n, 0.85, args.tol
    src, dst = graphgen.web_graph(n, seed=0, alpha=args.alpha, kmax=args.kmax)
    stats = graphgen.graph_stats(n, src, dst)
    g = di.Graph(n, src, dst)
    del src, dst
    if args.window_cfg:
        vals = [int(v) for v in args.window_cfg.split(",")]
        if di.di_graph_set_window(g.handle, *vals) != di.DI_OK:
            raise RuntimeError(di.di_last_error())
    X = torch.empty(n, dtype=torch.float64, device="cuda")
    opts = di.di_opts_default()
    opts.kernel = {"auto": di.DI_KERNEL_AUTO, "pull": di.DI_KERNEL_PULL, "push": di.DI_KERNEL_PUSH,
                   "window": di.DI_KERNEL_WINDOW}[args.kernel]
    # the move kernel DI_KERNEL_AUTO takes
    kind = {"auto": "window", "pull": "pull", "push": "push", "window": "window"}[args.kernel]
    opts.precision = {"fp64": di.DI_FP64, "fp32": di.DI_FP32, "fp32r": di.DI_FP32_REFINE}[args.precision]
    headline = (n == 1_000_000 and args.kmax == 500 and args.precision == "fp64"
                and args.alpha == 1.68 and args.kernel != "push")

    def solve():
        status, st = di.di_solve_dev(g.handle, None, d, tol, opts, X)
        if status != di.DI_OK:
            raise RuntimeError(f"{di.STATUS_NAMES.get(status)}: {di.di_last_error()}")
        return st

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    # what the first DI_KERNEL_AUTO solve tuned: the window configuration,
    # and whether the pull is faster on this graph
    tuning = di.di_graph_tuning(g.handle)
    if args.kernel == "auto":
        kind = tuning["kernel"]
    t0 = time.perf_counter()
    runs = [solve() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sec = wall / args.steps
    last = runs[-1]

    # Second pass, same workload: HIP events around every pull (or push)
    # launch give the dominant kernel's mean duration. Events add their own
    # stream packets, so they are kept out of the pass that gives `value`.
    opts.flags = di.DI_FLAG_KERNEL_TIMING
    torch.cuda.synchronize()
    runs = [solve() for _ in range(args.steps)]
    torch.cuda.synchronize()
    opts.flags = 0

    # method bytes (what DI-SOP itself moves: per link moved, per diffused
    # node, and the selection's pass over F and the node words) per launch
    move_bytes = sum(r.move_bytes for r in runs)
    move_secs = sum(r.move_seconds for r in runs)
    launches = sum(r.move_launches for r in runs)
    per_launch_bytes = move_bytes / max(launches, 1)
    per_launch_s = move_secs / max(launches, 1)
    achieved = per_launch_bytes / per_launch_s / 1e9 if per_launch_s > 0 else 0.0
    traffic = read_traffic(kind) if headline and kind in TRAFFIC else None
    edges = float(np.mean([r.edges_pushed for r in runs]))
    solutions = {f"DI-SOP {kind} fp64 (headline)": ("1m", "uniform", X.cpu().numpy())}
    # the same solve through the host-array entry (B and X cross PCIe)
    Xh = np.empty(n)
    di.di_solve(g.handle, None, d, tol, opts, Xh)
    t0 = time.perf_counter()
    for _ in range(5):
        status, _ = di.di_solve(g.handle, None, d, tol, opts, Xh)
        if status != di.DI_OK:
            raise RuntimeError(di.di_last_error())
    pcie_s = (time.perf_counter() - t0) / 5
    # an achievable copy rate on this device, beside the published peak:
    # 512 MiB read and 512 MiB written per copy, timed with events
    ca = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        cb.copy_(ca)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * ca.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb

    line = {
        "metric": "s to L1 resid\u22641e-9 and % HBM peak at N=1M; batched PPR solves/s, p50/p99 ms",
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32r": "f32 fluid, f64 residual"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"web graph N={n} seed 0, out-degree power law alpha={args.alpha} on "
                        f"[1,{args.kmax}], 15% dangling, 70% links within +-500, rest Zipf(1); "
                        f"d={d}, B=(1-d)/N, stop at sum|F|<={tol:g}, {args.precision}",
            "n": n, "links": int(stats.L), "dangling": int(stats.D),
            "kernel": kind,
        },
        "cycles": int(last.cycles),
        "nb_iter": float(last.nb_iter),
        "seconds_to_1e9": float(last.seconds_to_1e9),
        "tuning": tuning if args.kernel == "auto" else None,
        "gedges_per_s": edges / sec / 1e9,
        "bytes_per_edge": float(last.bytes_moved) / max(float(last.edges_pushed), 1.0),
        "host_arrays_s": pcie_s,
        "resid_l1": float(last.resid_l1),
        "err_bound": float(last.err_bound),
        "roofline": {
            "bound": "hbm",
            "kernel": {"window": "k_wcycle", "pull": "k_pull", "push": "k_push"}[kind]
                      + ("<double>" if args.precision == "fp64" else "<float>"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "method_bytes_per_launch": per_launch_bytes,
            "us_per_launch": per_launch_s * 1e6,
            "launches": launches,
            "traffic_over_method_bytes": (traffic / per_launch_bytes
                                          if traffic and per_launch_bytes > 0 else None),
            "achievable_copy_gbps": copy_gbps,
            "method_bytes": "per cycle N*(s+4) (selection reads F and the node word) + "
                            "(8+4s) per diffused node + (4+2s) per link moved, s = 8 (FP64); "
                            "the window launch selects and moves in one" if kind == "window" else
                            "(4+2s) per link moved, s = 8 (FP64)",
        },
    }
    if kind == "pull":
        # the pull reads every in-link each cycle: its dense scan, apart
        # from the method's bytes
        scan = float(stats.L) * 12.0 + n * 18.0
        line["roofline"]["pull_scan_model"] = {
            "bytes_per_launch": scan, "gbps": scan / per_launch_s / 1e9 if per_launch_s else 0.0,
            "frac": scan / per_launch_s / 1e9 / HBM_PEAK_GBS if per_launch_s else 0.0}
    if args.calibration_copy:
        # a write-only fill and a read-only sum of 1 GiB each (beyond the
        # 256 MB Infinity Cache), the last two kernels of the run
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        a.fill_(1.0)
        torch.cuda.synchronize()
        line["calibration_sum"] = float(a.sum().item())
        torch.cuda.synchronize()
        del a
    line["hbm_frac"] = line["roofline"]["frac"]
    if not args.no_extras and headline:
        sections = {
            "fp32_refine": lambda: fp32_refine_section(di, g, X, d, tol, solutions),
            "methods": lambda: methods_section(di, g, X, d, tol, solutions),
            "literal_alpha_1m": lambda: literal_alpha_section(di, graphgen, n, d, tol, args.kmax,
                                                              solutions),
            "config_10k": lambda: small_graph_section(di, graphgen, d, tol),
            "transposed_1m": lambda: transposed_section(di, graphgen, n, d, tol, args.alpha,
                                                        args.kmax),
            "dataset2_like": lambda: high_e_section(di, graphgen, d),
            "prefix_sweep": lambda: prefix_sweep_section(di, graphgen, n, d, tol, args.alpha,
                                                         args.kmax),
            "batched_ppr": lambda: batched_section(di, graphgen, g, n, d, tol, solutions),
            "serving": lambda: serving_section(di, graphgen, d, args.serve_seconds,
                                               args.serve_kmax),
        }
        for name, run in sections.items():
            if args.only is None or args.only == name:
                line[name] = run()
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(n, d, tol, args.cpu_seconds, args.alpha, args.kmax,
                                            solutions if headline else None,
                                            with_baselines=headline)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)
    g.close()


if __name__ == "__main__":
    main()
