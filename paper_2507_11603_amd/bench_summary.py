"""Render one bench.py JSON line as the markdown summary kept with the
profiles: the headline step, its kernels against their bounds, the counter
record it cites, the secondary figures, and the raw line.

    python -m paper_2507_11603_amd.bench_summary --bench-json LINE.json \\
        [--stats KERNEL_STATS.csv] --command "..." --out profiles/NAME.md
"""
from __future__ import annotations

import argparse
import csv
import json


def _line(path):
    with open(path) as f:
        for line in f:
            if line.startswith("{"):
                return json.loads(line)
    raise ValueError("no JSON line in %s" % path)


def render(d: dict, command: str, stats: str | None) -> str:
    c = d["config"]
    k = d["kernels"]
    r = d["roofline"]
    ph = d["path_hbm"]
    L = ["# %s" % c["workload"].split(" (")[0] + ", %d packets per step, %s: the default bench.py line"
         % (c["packets_per_step"], c["precision"]), "", "```", command, "```", "",
         "Device times from HIP events on the library stream; fields `%s`, knobs %s%s." % (
             c["fields"], json.dumps(c["knobs"]),
             " (autotuned on a %s-packet sample)" % c["autotuned"].get("sample") if c.get("autotuned") else ""), "",
         "* one step: %.2f s; **%.4g scatterings/s**, %.4g packets/s, %.1f scatterings per packet, "
         "longest history %d interactions" % (d["ms_per_step"] / 1e3, d["value"], d["packets_per_s"],
                                               d["scatterings_per_packet"], d["longest_history"]),
         "* cell visits: main %.4g, peel %.4g; whole path %.1f GB/s of algorithmic bytes (20 B per visit) "
         "= %.3f of 8 TB/s" % (ph["main_visits"], ph["peel_visits"], ph["achieved"], ph["frac"])]
    for name in ("transport", "tail", "peel_pass"):
        if name in k:
            L.append("* %s: %.0f ms over %d launches, %.4g visits, %.0f GB/s algorithmic = %.3f of HBM"
                     % (name, k[name]["ms"], k[name]["launches"], k[name]["visits"], k[name]["achieved_GBps"],
                        k[name]["hbm_frac"]))
    L.append("* presort of the queue: %.1f ms" % d.get("presort_ms", 0.0))
    def roof_line(title, r):
        traffic = ("%.4g B (%.2f of the algorithmic bytes)" % (r["traffic"], r["traffic_over_algorithmic"])
                   if r.get("traffic") else "not measured for these sources")
        src = ", from `%s`" % r["counters"] if r.get("counters") else ""
        if r["bound"] == "alu":
            rate = ("%.4g wave64 VALU instructions/s = %.3f of %.4g (VALU %.0f %% busy, %.0f %% lane utilisation)"
                    % (r["achieved"], r["frac"], r["peak"], r.get("valu_busy_pct") or 0.0,
                       r.get("valu_lane_util_pct") or 0.0) if r.get("achieved") else "VALU rate not measured")
            return ("* %s `%s`, bound by VALU issue: %s; average launch %.3f ms; algorithmic bytes %.1f GB/s "
                    "(%.3f of HBM); HBM traffic per launch %s%s"
                    % (title, r["kernel"], rate, r["avg_launch_ms"], r["hbm_achieved_GBps"], r["hbm_frac"],
                       traffic, src))
        return ("* %s `%s`, bound by HBM gathers: %.1f GB/s = %.3f of %.0f GB/s; average launch %.3f ms; "
                "HBM traffic per launch %s%s" % (title, r["kernel"], r["achieved"], r["frac"], r["peak"],
                                                 r["avg_launch_ms"], traffic, src))
    L.append(roof_line("roofline (dominant kernel)", r))
    if "hbm_gather" in d and d["hbm_gather"]["kernel"] != r["kernel"]:
        L.append(roof_line("HBM-gather roofline of the peel pass", d["hbm_gather"]))
    if "plain_fp64" in d:
        p = d["plain_fp64"]
        L.append("* plain FP64 path (%s): %.4g scatterings/s -> the persistent mixed path is %.0fx faster"
                 % (p["sample"], p["value"], d["speedup_vs_plain_fp64"]))
    if "cpu_baseline" in d:
        cb = d["cpu_baseline"]
        L.append("* CPU oracle on the host (%s, %d threads): %.4g scatterings/s; one thread %.4g (%s)"
                 % (cb["cpu_model"], cb["cores"], cb["value"], cb["one_core_value"], cb["sample"]))
    if "shell" in d:
        s = d["shell"]
        L.append("* %s: %d packets in %.2f s, %.4g scatterings/s, longest history %d; dominant `%s`"
                 % (s["workload"], s["packets"], s["seconds"], s["scatterings_per_s"], s["longest_history"],
                    s.get("dominant")))
    if "mg2" in d:
        g = d["mg2"]
        L.append("* %s, %d packets per velocity: %s" % (g["workload"], g["packets"], "; ".join(
            "%g km/s: %.3g packets/s, %.3g segments/s, F_blue/F_tot %.3f" % (
                r["v_max_kms"], r["packets_per_s"], r["segments_per_s"], r["blue_fraction"]) for r in g["runs"])))
    if "serving" in d:
        s = d["serving"]
        L.append("* serving: %d requests (+%d warm-up) at %.0f req/s: p50 %.1f ms, p99 %.1f ms; offered %.4g "
                 "packets/s, sustained %.4g" % (s["requests"], s["warmup_requests"], s["rate_hz"], s["p50_ms"],
                                                s["p99_ms"], s["offered_packets_per_s"],
                                                s["sustained_packets_per_s"]))
    if stats:
        with open(stats) as f:
            rows = list(csv.DictReader(f))
        L += ["", "rocprofv3 --stats over the whole command (every call, warm-up and secondary figures included):",
              "", "| Kernel | Calls | Total ms | Average ms | Share |", "|---|---|---|---|---|"]
        for row in rows[:8]:
            name = row["Name"].replace("void ", "").split("(")[0]
            L.append("| %s | %s | %.1f | %.3f | %s %% |" % (name, row["Calls"], float(row["TotalDurationNs"]) / 1e6,
                                                          float(row["AverageNs"]) / 1e6, row["Percentage"]))
    L += ["", "Raw line:", "", "```", json.dumps(d), "```"]
    return "\n".join(L) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--stats", default=None)
    ap.add_argument("--command", default="python bench.py")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    text = render(_line(a.bench_json), a.command, a.stats)
    with open(a.out, "w") as f:
        f.write(text)
    print(text[:2000])


if __name__ == "__main__":
    main()
