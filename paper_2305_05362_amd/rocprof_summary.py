"""Short text summaries of rocprofv3 output (CSV format) for the RAM kernels.

    python -m paper_2305_05362_amd.rocprof_summary stats DIR --command CMD --out FILE
        per-kernel dispatch count and durations from a --kernel-trace --stats
        run (DIR holds *_kernel_stats.csv);

    python -m paper_2305_05362_amd.rocprof_summary traffic --fetch DIR --write DIR
            --kernel SUBSTRING --copy-bytes N --command CMD --out FILE
        HBM bytes per dispatch of one kernel from two --pmc runs (FETCH_SIZE,
        then WRITE_SIZE; KiB per dispatch), each scaled by what the same
        counter reads for the largest plain device copy in the run (a copy of
        N bytes reads N and writes N bytes).

Both write a markdown file with a table and, for traffic, one fenced JSON
record that bench.py reads.  The record carries a digest of the kernel
sources; bench.py ignores it once the sources have changed.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _one(directory: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return hits[0]


def _short(name: str, width: int = 90) -> str:
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    cut = name.find("(ram::")
    if cut > 0:
        name = name[:cut]
    return name if len(name) <= width else name[:width - 3] + "..."


def stats(directory: str, command: str, out: str, top: int = 24) -> None:
    rows = list(csv.DictReader(open(_one(directory, "_kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel durations (rocprofv3 --kernel-trace --stats)", "",
             "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | % of GPU time |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    _write(out, lines)


def _counter(directory: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    vals = {}
    for r in csv.DictReader(open(_one(directory, "_counter_collection.csv"))):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _pick(vals, substring: str):
    names = [k for k in vals if substring in k]
    if len(names) != 1:
        raise ValueError(f"{substring!r} matches {len(names)} kernels: {names}")
    return names[0], vals[names[0]]


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: int,
            command: str, out: str, digest: str, units: int, unit_name: str,
            algorithmic_bytes_per_unit: float) -> dict:
    f = _counter(fetch_dir, "FETCH_SIZE")
    w = _counter(write_dir, "WRITE_SIZE")
    name, fk = _pick(f, kernel)
    _, wk = _pick(w, kernel)
    cf = max(f.get(COPY_KERNEL, [0.0]))
    cw = max(w.get(COPY_KERNEL, [0.0]))
    if cf <= 0 or cw <= 0:
        raise ValueError("no calibration copy in the counter runs")
    ff = cf * 1024.0 / copy_bytes
    wf = cw * 1024.0 / copy_bytes
    fetch = statistics.median(fk) * 1024.0 / ff
    write = statistics.median(wk) * 1024.0 / wf
    alg = algorithmic_bytes_per_unit * units
    rec = {"kernel": kernel, "kernel_name": _short(name, 200), "source_digest": digest,
           "dispatches": len(fk), "fetch_kib_median": statistics.median(fk),
           "write_kib_median": statistics.median(wk),
           "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": ff, "write_scale": wf,
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "traffic_bytes_per_launch": fetch + write,
           "units_per_launch": units, "unit": unit_name,
           "algorithmic_bytes_per_launch": alg,
           "traffic_over_algorithmic": (fetch + write) / alg}
    lines = ["# HBM traffic of one kernel (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
             "Commands (one counter per run):", "", "```", command, "```", "",
             f"Kernel: `{rec['kernel_name']}`, {len(fk)} dispatches per run.", "",
             "| quantity | FETCH_SIZE | WRITE_SIZE |", "|---|---:|---:|",
             f"| kernel, KiB per dispatch (median) | {rec['fetch_kib_median']:.0f} | "
             f"{rec['write_kib_median']:.0f} |",
             f"| plain copy of {copy_bytes} B, KiB | {cf:.0f} | {cw:.0f} |",
             f"| counter scale (copy KiB x 1024 / bytes) | {ff:.4f} | {wf:.4f} |",
             f"| kernel, bytes per dispatch after scaling | {fetch:.4g} | {write:.4g} |", "",
             f"Algorithmic bytes per launch: {alg:.4g} ({algorithmic_bytes_per_unit:g} B x "
             f"{units} {unit_name}); measured / algorithmic = "
             f"{rec['traffic_over_algorithmic']:.3f}.", "",
             "```json", json.dumps(rec), "```"]
    _write(out, lines)
    return rec


def read_traffic(path: str):
    """The JSON record of a traffic summary, or None."""
    try:
        text = open(path).read()
    except OSError:
        return None
    start = text.find("```json")
    if start < 0:
        return None
    end = text.find("```", start + 7)
    return json.loads(text[start + 7:end])


def _write(out: str, lines) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--units", type=int, required=True)
    t.add_argument("--unit-name", default="cells")
    t.add_argument("--bytes-per-unit", type=float, required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    a = p.parse_args(argv)
    if a.what == "stats":
        stats(a.dir, a.command, a.out)
    else:
        from .build import kernel_digest
        rec = traffic(a.fetch, a.write, a.kernel, a.copy_bytes, a.command, a.out,
                      kernel_digest(a.kernel), a.units, a.unit_name, a.bytes_per_unit)
        json.dump(rec, sys.stdout)
        print()


if __name__ == "__main__":
    main()
