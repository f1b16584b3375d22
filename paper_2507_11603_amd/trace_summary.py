"""Summarise a rocprofv3 kernel trace of one bench.py command.

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o t -- python3 bench.py ...
    python -m paper_2507_11603_amd.trace_summary --trace DIR --bench-json LINE.json \\
        --first-call W --calls K --out profiles/NAME.md

Every thor_transport call ends with one k_spec_fold dispatch, so the
dispatches between two of them belong to one call.  The summary lists, for
calls [first_call, first_call + calls) (the timed steps of the bench: the
warm-up calls come first), every kernel's dispatch count, total and average
duration from the trace, and, when the bench line is given, the dominant
kernel's average launch time that bench.py measured with HIP events, so the
two can be compared.  The whole trace's per-kernel table follows.
`--first-call -1` picks the longest call instead.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os


def _load(trace_dir: str):
    path = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    if not path:
        raise FileNotFoundError("no kernel_trace.csv under %s" % trace_dir)
    with open(path[0]) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return rows, path[0]


def _short(name: str) -> str:
    name = name.split("(")[0] if name.startswith("void ") else name
    return name.replace("void ", "")[:70]


def _table(rows):
    agg = collections.OrderedDict()
    for r in rows:
        k = _short(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += d
    return sorted(agg.items(), key=lambda kv: -kv[1][1])


def summarise(trace_dir: str, first_call: int, calls: int, bench: dict | None, command: str) -> str:
    rows, path = _load(trace_dir)
    groups, cur = [], []
    for r in rows:
        cur.append(r)
        if "k_spec_fold" in r["Kernel_Name"]:
            groups.append(cur)
            cur = []
    if first_call < 0:
        # the longest call (the timed 1e8-packet step of the default bench,
        # whose autotuner and warm-up calls come first)
        span = [sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in g) for g in groups]
        first_call = max(range(len(groups)), key=lambda i: span[i])
        calls = 1
    sel = [r for g in groups[first_call:first_call + calls] for r in g]
    lines = ["Command (from the repository root on the GPU host):", "", "```", command, "```", "",
             "Trace: `%s` (%d dispatches, %d thor_transport calls).  Calls %d..%d are the timed steps."
             % (os.path.basename(path), len(rows), len(groups), first_call, first_call + calls - 1), "",
             "| Kernel (timed calls) | Dispatches | Total ms | Average ms |", "|---|---|---|---|"]
    for k, (n, ms) in _table(sel):
        lines.append("| %s | %d | %.2f | %.3f |" % (k, n, ms, ms / n))
    if bench:
        roof = bench.get("roofline", {})
        if roof.get("bound") == "alu":
            rate = ("%.4g wave64 VALU instructions/s = %.3f of %.4g" % (roof["achieved"], roof["frac"], roof["peak"])
                    if roof.get("achieved") else "VALU rate not measured")
            lines += ["", "bench.py (HIP events on the library stream) for the dominant kernel `%s` (bound by "
                      "VALU issue): %d launches, average %.3f ms, %s." % (roof.get("kernel"), roof.get("launches", 0),
                                                                        roof.get("avg_launch_ms", 0.0), rate)]
        else:
            lines += ["", "bench.py (HIP events on the library stream) for the dominant kernel `%s`: %d launches, "
                      "average %.3f ms, %.4g algorithmic bytes per launch, %.1f GB/s = %.3f of %.0f GB/s."
                      % (roof.get("kernel"), roof.get("launches", 0), roof.get("avg_launch_ms", 0.0),
                         roof.get("algorithmic_bytes_per_launch", 0.0), roof.get("achieved", 0.0),
                         roof.get("frac", 0.0), roof.get("peak", 0.0))]
        kshort = (roof.get("kernel") or "").split("<")[0]
        tr = [(n, ms) for k, (n, ms) in _table(sel) if kshort and kshort in k]
        if tr:
            n = sum(t[0] for t in tr)
            ms = sum(t[1] for t in tr)
            lines.append("Trace for the same kernel in the timed calls: %d dispatches, average %.3f ms "
                         "(ratio to bench.py's average: %.3f)."
                         % (n, ms / n, (ms / n) / max(roof.get("avg_launch_ms", 1e-9), 1e-9)))
    lines += ["", "Whole trace:", "", "| Kernel | Dispatches | Total ms | Average ms |", "|---|---|---|---|"]
    for k, (n, ms) in _table(rows)[:16]:
        lines.append("| %s | %d | %.2f | %.3f |" % (k, n, ms, ms / n))
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--bench-json", default="")
    ap.add_argument("--first-call", type=int, default=1)
    ap.add_argument("--calls", type=int, default=1)
    ap.add_argument("--command", default="")
    ap.add_argument("--title", default="Kernel trace")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    bench = None
    if a.bench_json:
        with open(a.bench_json) as f:
            for line in f:
                line = line.strip()
                if line.startswith("{"):
                    bench = json.loads(line)
    text = "# %s\n\n" % a.title + summarise(a.trace, a.first_call, a.calls, bench, a.command)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
