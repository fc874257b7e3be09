"""Summaries of rocprofv3 output for the solver's kernels.

``python -m paper_2512_16889_amd.prof_summary stats <kernel_stats.csv>``
prints a markdown table of the per-kernel dispatch statistics;
``... launches <kernel_trace.csv> [top]`` the same from the trace, per kernel
and launch grid.

``python -m paper_2512_16889_amd.prof_summary traffic <pmc_fetch.csv>
<pmc_write.csv> <copy_fetch.csv> <copy_write.csv> <copy_bytes>`` prints, as
JSON, the HBM bytes per dispatch of every kernel in the first two arguments
(FETCH_SIZE and WRITE_SIZE, KiB per dispatch; each may be a comma-separated
list of files, e.g. runs with different tile variants forced), each scaled by
what the same counter reads for a plain device copy of ``copy_bytes`` bytes
each way, and the sha256 of the kernel sources they were taken from.
"""
from __future__ import annotations

import csv
import json
import statistics
import sys


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def stats_table(path, top=16):
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def launch_table(path, top=24, min_us=0.0):
    """Markdown table of a kernel trace grouped by kernel and launch grid, so
    that batched and per-solve launches of one kernel are told apart."""
    groups = {}
    for r in _rows(path):
        key = (r["Kernel_Name"], int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in groups.values())
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    out = ["| kernel | grid | calls | avg us | min us | max us | % of time |", "|---|---|---|---|---|---|---|"]
    for (name, gx, gy), d in rows[:top]:
        avg = statistics.mean(d)
        if avg < min_us:
            continue
        out.append(f"| `{name[:80]}` | {gx} x {gy} | {len(d)} | {avg:.1f} | {min(d):.1f} | {max(d):.1f} | "
                   f"{100.0 * sum(d) / total:.2f} |")
    return "\n".join(out)


def _per_kernel(paths, counter):
    acc = {}
    for path in paths.split(","):
        for r in _rows(path):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
    return acc


def _copy_scale(path, counter, copy_bytes):
    vals = _per_kernel(path, counter)
    big = [v for name, vs in vals.items() if "copyBuffer" in name for v in vs if v > 0.25 * copy_bytes]
    return copy_bytes / statistics.median(big)


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes):
    from .build import source_hash
    fs = _copy_scale(copy_fetch_csv, "FETCH_SIZE", copy_bytes)
    ws = _copy_scale(copy_write_csv, "WRITE_SIZE", copy_bytes)
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    kern = {}
    for name in sorted(set(f) & set(w)):
        if "swf::" not in name:
            continue
        kern[name] = {"dispatches": len(f[name]), "fetch_bytes": statistics.mean(f[name]) * fs,
                      "write_bytes": statistics.mean(w[name]) * ws}
    return {"kernel_source_sha256": source_hash(), "fetch_scale": fs, "write_scale": ws, "kernels": kern}


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats_table(sys.argv[2]))
    elif sys.argv[1] == "launches":
        print(launch_table(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 24))
    elif sys.argv[1] == "traffic":
        print(json.dumps(traffic(*sys.argv[2:6], float(sys.argv[6])), indent=1))
