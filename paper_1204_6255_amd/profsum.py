"""Summaries of rocprofv3 output for the committed profiles/ files.

    python -m paper_1204_6255_amd.profsum trace OUT_NAME DIR "<title>" "<command>"

writes profiles/OUT_NAME: the per-kernel table of a `--kernel-trace
--stats` run (csv, output name `run`).

    python -m paper_1204_6255_amd.profsum traffic OUT_NAME KERNEL SOURCE FETCH_DIR WRITE_DIR \
        "<title>" "<fetch command>" "<write command>"

writes profiles/OUT_NAME: HBM bytes per launch of KERNEL (short name) from
`--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the benchmark with
--calibration-copy, each counter scaled by what it reads for a 1 GiB
read-only sum and a 1 GiB write-only fill, with the raw readings.

    python -m paper_1204_6255_amd.profsum counters OUT_NAME DIR "<command>" [DIR "<command>" ...]

writes profiles/OUT_NAME: the mean per dispatch of every counter that
`--pmc` runs of the benchmark collected for the cycle kernels.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def short(name: str) -> str:
    return name.replace("di::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def kernel_stats(d: str):
    with open(os.path.join(d, "run_kernel_stats.csv")) as f:
        return list(csv.DictReader(f))


CAL_KIB = 1024 * 1024  # bytes (in KiB) written by the calibration fill and read by its sum


def calibration_kib(d: str, kind: str) -> float:
    """The counter value of the run's last calibration dispatch of one kind:
    'fill' (torch's fill of 1 GiB, write-only) or 'sum' (torch's reduction
    over the same 1 GiB, read-only), which bench.py --calibration-copy runs
    after everything else."""
    last_id, value = -1, None
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            hit = ("FillFunctor" in name) if kind == "fill" else ("reduce_kernel" in name)
            if hit and int(r["Dispatch_Id"]) > last_id:
                last_id, value = int(r["Dispatch_Id"]), float(r["Counter_Value"])
    if value is None:
        raise SystemExit(f"no {kind} calibration dispatch in {d}")
    return value


def counters(d: str):
    agg = collections.defaultdict(list)
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


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
            if k.startswith(("k_pull", "k_select", "k_wcycle", "k_wfold")):
                for c, v in sorted(agg[k].items()):
                    lines.append(f"{k}\t{c}\t{sum(v) / len(v):.0f}\tdispatches={len(v)}")
    with open(os.path.join(PROFILES, out_name), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic_main(argv):
    """traffic OUT_NAME KERNEL SOURCE FETCH_DIR WRITE_DIR TITLE FETCH_CMD WRITE_CMD:
    HBM bytes per launch of one kernel (its short name, e.g.
    k_wcycle<double>). FETCH_SIZE is scaled by what it reads for the
    read-only 1 GiB sum, WRITE_SIZE by what it reads for the write-only 1 GiB
    fill; the raw readings are listed too. SOURCE is the kernel's source
    file, whose hash bench.py checks before it reports the figure."""
    out_name, kernel, source, fetch_dir, write_dir, title, fetch_cmd, write_cmd = argv[:8]
    fe, wr = counters(fetch_dir), counters(write_dir)
    sum_fetch, fill_write = calibration_kib(fetch_dir, "sum"), calibration_kib(write_dir, "fill")
    fill_fetch, sum_write = calibration_kib(fetch_dir, "fill"), calibration_kib(write_dir, "sum")
    ff = CAL_KIB / sum_fetch
    fw = CAL_KIB / fill_write
    name = [k for k in fe if short(k) == kernel][0]
    f_kib = sum(fe[name]) / len(fe[name])
    w_kib = sum(wr[name]) / len(wr[name])
    with open(os.path.join(ROOT, source), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    lines = [
        f"# HBM traffic of {kernel} per launch, {title}",
        f"# fetch command: {fetch_cmd}",
        f"# write command: {write_cmd}",
        "# FETCH_SIZE / WRITE_SIZE are KiB per dispatch. FETCH_SIZE is scaled so that it reads",
        "# 1 GiB for torch's sum over a 1 GiB tensor (read-only), WRITE_SIZE so that it reads",
        "# 1 GiB for torch's fill of the same tensor (write-only); both run last in the command",
        "# and are four times the 256 MB Infinity Cache.",
        f"calibration_sum_fetch_kib: {sum_fetch:.1f}",
        f"calibration_sum_write_kib: {sum_write:.1f}",
        f"calibration_fill_fetch_kib: {fill_fetch:.1f}",
        f"calibration_fill_write_kib: {fill_write:.1f}",
        f"fetch_scale: {ff:.4f}",
        f"write_scale: {fw:.4f}",
        f"dispatches: {len(fe[name])}",
        f"fetch_kib_mean: {f_kib:.1f}",
        f"write_kib_mean: {w_kib:.1f}",
        f"traffic_bytes_per_launch: {(f_kib * ff + w_kib * fw) * 1024:.0f}",
        f"kernel_source: {source}",
        f"kernel_source_sha256_16: {sha}",
    ]
    for k in sorted(fe, key=short):
        w = wr.get(k, [0.0])
        lines.append(f"# other: {short(k)} fetch_kib_mean={sum(fe[k]) / len(fe[k]):.1f} "
                     f"write_kib_mean={sum(w) / len(w):.1f} dispatches={len(fe[k])}")
    with open(os.path.join(PROFILES, out_name), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_main(argv):
    """trace OUT_NAME DIR TITLE CMD [AFTER_KERNEL]: the per-kernel table of a
    `--kernel-trace --stats` run. With AFTER_KERNEL (a short name, e.g.
    k_pull<double>), a second table covers only the dispatches that start
    after that kernel's last dispatch (for instance after a tuner that times
    that kernel last), and lists apart those under 12 us (launches that
    return at the stop test)."""
    out_name, d, title, cmd = argv[:4]
    after = argv[4] if len(argv) > 4 else None
    lines = [f"# rocprofv3 kernel summary: {title}", f"# command: {cmd}",
             "# columns: kernel, calls, total_us, average_us, min_us, max_us, percent"]
    for r in kernel_stats(d):
        lines.append(f"{short(r['Name'])}\t{r['Calls']}\t{float(r['TotalDurationNs']) / 1e3:.1f}\t"
                     f"{float(r['AverageNs']) / 1e3:.2f}\t{float(r['MinNs']) / 1e3:.2f}\t"
                     f"{float(r['MaxNs']) / 1e3:.2f}\t{float(r['Percentage']):.1f}")
    if after:
        with open(os.path.join(d, "run_kernel_trace.csv")) as f:
            rows = list(csv.DictReader(f))
        t0 = max(int(r["End_Timestamp"]) for r in rows if short(r["Kernel_Name"]) == after)
        per = collections.defaultdict(list)
        for r in rows:
            if int(r["Start_Timestamp"]) > t0:
                per[short(r["Kernel_Name"])].append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        lines.append(f"# dispatches after the last {after}: kernel, calls, average_us, min_us, "
                     "max_us; then the same over the calls of at least 12 us")
        for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            full = [x for x in v if x >= 12.0]
            line = (f"{k}\t{len(v)}\t{sum(v) / len(v):.2f}\t{min(v):.2f}\t{max(v):.2f}")
            if full:
                line += (f"\t| {len(full)}\t{sum(full) / len(full):.2f}\t{min(full):.2f}"
                         f"\t{max(full):.2f}")
            lines.append(line)
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
        raise SystemExit(__doc__)
