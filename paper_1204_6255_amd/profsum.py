"""Summaries of rocprofv3 output for the committed profiles/ files.

    python -m paper_1204_6255_amd.profsum TRACE_DIR FETCH_DIR WRITE_DIR \
        "<trace command>" "<fetch command>" "<write command>"

TRACE_DIR holds a `--kernel-trace --stats` run of the benchmark (csv,
output name `run`); FETCH_DIR / WRITE_DIR hold `--pmc FETCH_SIZE` and
`--pmc WRITE_SIZE` runs of it with --calibration-copy. Writes
profiles/di_sop_f64_n1m_kernels.txt (per-kernel durations) and
profiles/k_pull_f64_n1m_traffic.txt (HBM bytes per pull launch, with each
counter scaled by what it reads for the 256 MiB calibration copy).

    python -m paper_1204_6255_amd.profsum counters OUT_NAME DIR "<command>" [DIR "<command>" ...]

writes profiles/OUT_NAME: the mean per dispatch of every counter that
`--pmc` runs of the benchmark collected for the pull and the select.

    python -m paper_1204_6255_amd.profsum trace OUT_NAME DIR "<title>" "<command>"

writes profiles/OUT_NAME: the per-kernel table of any `--kernel-trace
--stats` run (csv, output name `run`).

    python -m paper_1204_6255_amd.profsum traffic OUT_NAME KERNEL FETCH_DIR WRITE_DIR "<title>" \
        "<fetch command>" "<write command>"

writes profiles/OUT_NAME: HBM bytes per launch of KERNEL (short name) from
`--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs with --calibration-copy.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1204_6255_amd", "csrc", "di_kernels.hip")
COPY_KIB = 256 * 1024  # read and written by the calibration copy


def short(name: str) -> str:
    return name.replace("di::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def kernel_stats(d: str):
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        return list(csv.DictReader(f))


def calibration_kib(d: str) -> float:
    """The counter value of the run's last copy dispatch: the calibration copy
    bench.py makes after its timed region (earlier copies are uploads)."""
    last_id, value = -1, None
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if short(r["Kernel_Name"]) == "__amd_rocclr_copyBuffer" and int(r["Dispatch_Id"]) > last_id:
                last_id, value = int(r["Dispatch_Id"]), float(r["Counter_Value"])
    return value


def counters(d: str):
    agg = collections.defaultdict(list)
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def main(argv):
    trace_dir, fetch_dir, write_dir, trace_cmd, fetch_cmd, write_cmd = argv[:6]
    out = ["# rocprofv3 kernel summary: DI-SOP FP64 on the N=1M web graph (benchmark workload)",
           f"# command: {trace_cmd}",
           "# columns: kernel, calls, total_us, average_us, min_us, max_us, percent"]
    for r in kernel_stats(trace_dir):
        out.append(f"{short(r['Name'])}\t{r['Calls']}\t{float(r['TotalDurationNs']) / 1e3:.1f}\t"
                   f"{float(r['AverageNs']) / 1e3:.2f}\t{float(r['MinNs']) / 1e3:.2f}\t"
                   f"{float(r['MaxNs']) / 1e3:.2f}\t{float(r['Percentage']):.1f}")
    with open(os.path.join(PROFILES, "di_sop_f64_n1m_kernels.txt"), "w") as f:
        f.write("\n".join(out) + "\n")
    fe, wr = counters(fetch_dir), counters(write_dir)
    cf, cw = calibration_kib(fetch_dir), calibration_kib(write_dir)
    ff = COPY_KIB / cf
    fw = COPY_KIB / cw
    pull = [k for k in fe if short(k) == "k_pull<double>"][0]
    f_kib = sum(fe[pull]) / len(fe[pull])
    w_kib = sum(wr[pull]) / len(wr[pull])
    with open(KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    lines = [
        "# HBM traffic of k_pull<double> per launch, DI-SOP FP64 on the N=1M web graph "
        "(benchmark workload)",
        f"# fetch command: {fetch_cmd}",
        f"# write command: {write_cmd}",
        "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by the factor that makes",
        "# the same counter read 256 MiB for the 256 MiB torch copy (__amd_rocclr_copyBuffer)",
        "# run last in the same command (--calibration-copy).",
        f"copy_fetch_kib: {cf:.1f}",
        f"copy_write_kib: {cw:.1f}",
        f"fetch_scale: {ff:.4f}",
        f"write_scale: {fw:.4f}",
        f"pull_dispatches: {len(fe[pull])}",
        f"pull_fetch_kib_mean: {f_kib:.1f}",
        f"pull_write_kib_mean: {w_kib:.1f}",
        f"traffic_bytes_per_launch: {(f_kib * ff + w_kib * fw) * 1024:.0f}",
        f"kernel_source_sha256_16: {sha}",
    ]
    for k in sorted(fe, key=short):
        w = wr.get(k, [0.0])
        lines.append(f"# other: {short(k)} fetch_kib_mean={sum(fe[k]) / len(fe[k]):.1f} "
                     f"write_kib_mean={sum(w) / len(w):.1f} dispatches={len(fe[k])}")
    with open(os.path.join(PROFILES, "k_pull_f64_n1m_traffic.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(out))
    print("\n".join(lines))


def counters_main(argv):
    """counters OUT_NAME DIR CMD [DIR CMD ...]: mean value per dispatch of
    every counter collected for k_pull<double> and k_select, one line each."""
    out_name, rest = argv[0], argv[1:]
    lines = ["# rocprofv3 counters per dispatch (mean over dispatches), DI-SOP FP64 on the N=1M "
             "web graph (benchmark workload)"]
    for d, cmd in zip(rest[0::2], rest[1::2]):
        lines.append(f"# command: {cmd}")
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                agg[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        for k in sorted(agg):
            if k.startswith("k_pull") or k.startswith("k_select"):
                for c, v in sorted(agg[k].items()):
                    lines.append(f"{k}\t{c}\t{sum(v) / len(v):.0f}\tdispatches={len(v)}")
    with open(os.path.join(PROFILES, out_name), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_main(argv):
    """traffic OUT_NAME KERNEL FETCH_DIR WRITE_DIR TITLE FETCH_CMD WRITE_CMD:
    HBM bytes per launch of one kernel (its short name, e.g. k_pull<float>),
    each counter scaled by what it reads for the calibration copy."""
    out_name, kernel, fetch_dir, write_dir, title, fetch_cmd, write_cmd = argv[:7]
    fe, wr = counters(fetch_dir), counters(write_dir)
    cf, cw = calibration_kib(fetch_dir), calibration_kib(write_dir)
    ff = COPY_KIB / cf
    fw = COPY_KIB / cw
    name = [k for k in fe if short(k) == kernel][0]
    f_kib = sum(fe[name]) / len(fe[name])
    w_kib = sum(wr[name]) / len(wr[name])
    lines = [
        f"# HBM traffic of {kernel} per launch, {title}",
        f"# fetch command: {fetch_cmd}",
        f"# write command: {write_cmd}",
        "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled by the factor that makes",
        "# the same counter read 256 MiB for the 256 MiB torch copy run last in the same command.",
        f"copy_fetch_kib: {cf:.1f}",
        f"copy_write_kib: {cw:.1f}",
        f"fetch_scale: {ff:.4f}",
        f"write_scale: {fw:.4f}",
        f"dispatches: {len(fe[name])}",
        f"fetch_kib_mean: {f_kib:.1f}",
        f"write_kib_mean: {w_kib:.1f}",
        f"traffic_bytes_per_launch: {(f_kib * ff + w_kib * fw) * 1024:.0f}",
    ]
    with open(os.path.join(PROFILES, out_name), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_main(argv):
    """trace OUT_NAME DIR TITLE CMD: the per-kernel table of a
    `--kernel-trace --stats` run."""
    out_name, d, title, cmd = argv[:4]
    lines = [f"# rocprofv3 kernel summary: {title}", f"# command: {cmd}",
             "# columns: kernel, calls, total_us, average_us, min_us, max_us, percent"]
    for r in kernel_stats(d):
        lines.append(f"{short(r['Name'])}\t{r['Calls']}\t{float(r['TotalDurationNs']) / 1e3:.1f}\t"
                     f"{float(r['AverageNs']) / 1e3:.2f}\t{float(r['MinNs']) / 1e3:.2f}\t"
                     f"{float(r['MaxNs']) / 1e3:.2f}\t{float(r['Percentage']):.1f}")
    with open(os.path.join(PROFILES, out_name), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    if sys.argv[1:2] == ["counters"]:
        counters_main(sys.argv[2:])
    elif sys.argv[1:2] == ["trace"]:
        trace_main(sys.argv[2:])
    elif sys.argv[1:2] == ["traffic"]:
        traffic_main(sys.argv[2:])
    else:
        main(sys.argv[1:])
