#!/usr/bin/env python3
"""Summaries of rocprofv3 output for profiles/ (runs on the CPU, after a profiled run).

    python profile_summary.py stats <rocprof-output-dir> --command "<cmd>" --out profiles/X.md
        per-kernel call count and durations from the --stats CSV (kernel_stats.csv)

    python profile_summary.py traffic --fetch <dir> --write <dir> --precision f32 \\
        --workload tracking_T2^20 --command-fetch "<cmd>" --command-write "<cmd>" \\
        --out profiles/X.md
        HBM bytes per launch of the benchmark's kernels from two counter runs
        (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by the same
        counter's reading for the library's plain copy kernel k_copy16 of known
        size (256 MiB read + 256 MiB written per dispatch, launched by bench.py).
        The result is merged into profiles/traffic.json under
        "<kernel>|<workload>|<precision>", with the hash of the kernel sources it
        was measured on; bench.py reports it only while that hash still matches.

Only reads CSV files that rocprofv3 wrote (--output-format csv).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "k_copy16"
COPY_BYTES = 256 << 20
# benchmark kernel key -> substring of the (demangled) rocprofv3 kernel name
KERNELS = {"k_prepare": "k_prepare", "k_filter": "k_filter", "k_rts": "k_rts",
           "k_twofilter": "k_twofilter"}


def _find(d: str, suffix: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def _short(name: str) -> str:
    base = name.split("(")[0]
    for key in (COPY_KERNEL,) + tuple(KERNELS.values()):
        if key in base:
            return base.replace("void ", "").strip()
    return base.strip()


def cmd_stats(a) -> int:
    files = _find(a.dir, "kernel_stats.csv")
    if not files:
        print("no kernel_stats.csv under", a.dir, file=sys.stderr)
        return 1
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append(r)
    lines = ["# rocprofv3 kernel statistics: %s" % a.title, "",
             "Command (from the repository root):", "", "```", a.command, "```", "",
             "| Kernel | Calls | Average (us) | Min (us) | Max (us) | Total (%) |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    if a.note:
        lines += ["", a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def _counter_means(d: str, counter: str) -> dict[str, list[float]]:
    files = _find(d, "counter_collection.csv")
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    vals: dict[str, list[float]] = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _source_hash() -> str:
    sys.path.insert(0, ROOT)
    import bench  # noqa: E402  (hash helper only; bench.main() is not run)
    return bench.kernel_source_hash()


def cmd_traffic(a) -> int:
    fetch = _counter_means(a.fetch, "FETCH_SIZE")
    write = _counter_means(a.write, "WRITE_SIZE")

    def pick(vals, sub):
        xs = [v for k, vs in vals.items() if sub in k.split("(")[0] for v in vs]
        return statistics.median(xs) if xs else None

    cf, cw = pick(fetch, COPY_KERNEL), pick(write, COPY_KERNEL)
    if not cf or not cw:
        raise SystemExit("the copy kernel %s was not found in both runs" % COPY_KERNEL)
    kf = COPY_BYTES / (cf * 1024.0)
    kw = COPY_BYTES / (cw * 1024.0)
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    h = _source_hash()
    lines = ["# HBM traffic per launch (rocprofv3 counters): %s, %s" % (a.workload, a.precision), "",
             "Commands (from the repository root):", "", "```", a.command_fetch, a.command_write,
             "```", "",
             "Calibration: `%s` copies %d MiB per dispatch (reads and writes exactly that); "
             "it read FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB, so the scale factors are "
             "%.4f (fetch) and %.4f (write)." % (COPY_KERNEL, COPY_BYTES >> 20, cf, cw, kf, kw), "",
             "| Kernel | FETCH_SIZE (KiB, median) | WRITE_SIZE (KiB, median) | HBM bytes per launch "
             "(scaled) |", "|---|---|---|---|"]
    for key, sub in KERNELS.items():
        f_, w_ = pick(fetch, sub), pick(write, sub)
        if f_ is None or w_ is None:
            continue
        total = f_ * 1024.0 * kf + w_ * 1024.0 * kw
        data["%s|%s|%s" % (key, a.workload, a.precision)] = {
            "bytes_per_launch": total, "fetch_kib": f_, "write_kib": w_,
            "fetch_scale": kf, "write_scale": kw, "source_hash": h}
        lines.append("| `%s` | %.0f | %.0f | %.4g |" % (key, f_, w_, total))
    lines += ["", "Kernel-source hash at measurement: `%s`." % h]
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--precision", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    return cmd_stats(a) if a.cmd == "stats" else cmd_traffic(a)


if __name__ == "__main__":
    sys.exit(main())
