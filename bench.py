"""Benchmark of the Lyman-alpha packet-transport hot path on one MI355X.

One step = one whole pass of the hot path over one batch: emit 1e6 packets
from the central source of the 128^3 expanding-shell grid, march them with
the Voigt cross-section in the gas frame, scatter (resonant and dust), peel
off to the +z cube and bin the escapes.  Inputs are resident in HBM before
the timed region (the grid is loaded once, untimed).

Prints one JSON line (see the keys below).  `value` is photon scatterings
per second (resonant + dust) of the persistent mixed-precision path; the
plain one-launch-per-batch FP64 path is timed on the same GPU beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
BYTES_PER_VISIT = 20.0         # (vx, vy, vz, n_HI, T) float32 per cell visit


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=1_000_000)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--path", default="persistent", choices=["persistent", "plain"])
    ap.add_argument("--plain-steps", type=int, default=2, help="steps of the plain FP64 path (0: skip)")
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--turn-visits", type=int, default=0)
    ap.add_argument("--inline-peel", type=int, default=0, help="march peel rays in the scattering lane")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=400000, help="packets of the oracle sample")
    ap.add_argument("--autotune", type=int, default=1, help="pick launch knobs with the autotuner")
    ap.add_argument("--serving", type=int, default=300, help="requests of the serving stream (0: skip)")
    ap.add_argument("--serving-warmup", type=int, default=60)
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--web-grid", type=int, default=0,
                    help="also measure the cosmic-web box at this grid size (fields generated on the GPU)")
    ap.add_argument("--web-packets", type=int, default=100_000)
    ap.add_argument("--web-fields", default="gpu", choices=["gpu", "cpu"],
                    help="make the web fields with torch on the GPU or with numpy on the host")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (PMC calibration)")
    return ap.parse_args()


def measured_traffic(a):
    """HBM-side bytes per launch of the timed kernel from the committed counter
    record (two rocprofv3 passes, calibrated on a plain copy), or None when the
    record is missing, was taken on another workload, or the kernel sources have
    changed since."""
    from paper_2507_11603_amd import pmc_summary
    path = os.path.join(ROOT, "profiles", "shell%d_traffic.json" % a.grid)
    if a.path != "persistent" or a.precision != "mixed" or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != pmc_summary.source_hash():
        return None
    per_batch = rec["fetch_bytes_per_batch"] + rec["write_bytes_per_batch"]
    return {"bytes": per_batch * a.steps, "fetch_bytes": rec["fetch_bytes_per_batch"] * a.steps,
            "write_bytes": rec["write_bytes_per_batch"] * a.steps,
            "over_algorithmic": rec["traffic_over_algorithmic"], "record": os.path.relpath(path, ROOT)}


def run_steps(T, wl, n, steps, first_id, **kw):
    """Queue `steps` batches of n packets (distinct photon ids) and transport
    them with one thor_transport call: the persistent path runs all batches
    in one launch of resident waves, the plain path one launch per batch."""
    import torch
    T.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        T.emit(wl["src"], n, first_id + s * n)
    code, st = T.transport(wl["opts"], **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert st["emitted"] == n * steps
    return dt, st


def cpu_baseline(wl, n):
    import oracle
    workers = min(16, os.cpu_count() or 1)
    oracle.build()
    t0 = time.perf_counter()
    r = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, n, workers=workers)
    dt = time.perf_counter() - t0
    scat = r["stats"]["n_res"] + r["stats"]["n_dust"]
    return dict(value=scat / dt, unit="scatterings/s", cores=workers, kind="oracle",
                sample="%d packets of the same 128^3 shell workload (ids 0..%d, seed 2), "
                       "%d scatterings in %.1f s over %d processes" % (n, n - 1, scat, dt, workers),
                packets_per_s=n / dt)


def serving(a, kw):
    """Open-loop stream of shell-model requests through the continuous-batching
    server: p50/p99 latency (completion - arrival) and sustained throughput."""
    import workloads as W
    from paper_2507_11603_amd import serve
    stream = W.request_stream(a.serving + a.serving_warmup, rate_hz=a.serving_rate)
    srv = serve.ShellServer(precision=a.precision, step_events=64,
                            waves_per_cu=kw.get("waves_per_cu", 0), visits_per_turn=kw.get("visits_per_turn", 0))
    try:
        r = srv.run_stream(stream, warmup=a.serving_warmup)
    finally:
        srv.close()
    pk = sum(q["n_packets"] for q in stream)
    span = stream[-1]["t_arrival"] - stream[0]["t_arrival"]
    return {"requests": a.serving, "warmup_requests": a.serving_warmup, "rate_hz": a.serving_rate,
            "p50_ms": r["p50_s"] * 1e3, "p99_ms": r["p99_s"] * 1e3,
            "offered_packets_per_s": pk / span, "sustained_packets_per_s": pk / r["wall_s"],
            "sustained_scatterings_per_s": r["scatterings"] / r["wall_s"], "wall_s": r["wall_s"],
            "steps": r["steps"], "budget_deferrals": r["deferrals"], "graph_steps": True}


def web_box(a, kw):
    """Cosmic-web box (n_HI^2 thermal emission, x_crit = 3, three observers):
    cell visits per second and the HBM-gather fraction at 20 B per visit."""
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    f = W.web_fields_torch(a.web_grid) if a.web_fields == "gpu" else W.web_fields(a.web_grid)
    wl = W.web(n_grid=a.web_grid, fields=f)
    T = thor.Transport(0)
    try:
        T.load(wl["geom"])
        del f, wl["geom"]["n_HI_field"], wl["geom"]["T_field"], wl["geom"]["vx"], wl["geom"]["vy"], wl["geom"]["vz"]
        if a.web_fields == "gpu":
            torch.cuda.empty_cache()
        wkw = {k: v for k, v in kw.items() if k != "visits_per_turn"}
        run_steps(T, wl, a.web_packets // 10, 1, 10**13, **wkw)           # warm-up (CDF, caches)
        dt, st = run_steps(T, wl, a.web_packets, 1, 0, **wkw)
    finally:
        T.close()
    visits = st["main_visits"] + st["peel_visits"]
    ks = st["kernel_ms"] / 1e3
    ach = BYTES_PER_VISIT * visits / ks / 1e9
    return {"grid": a.web_grid, "packets": a.web_packets, "seconds": dt, "kernel_ms": st["kernel_ms"],
            "scatterings_per_s": (st["n_res"] + st["n_dust"]) / dt, "packets_per_s": st["emitted"] / dt,
            "main_visits": st["main_visits"], "peel_visits": st["peel_visits"],
            "cell_visits_per_s": visits / ks,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": None}}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import workloads as W
    wl = W.shell(n_grid=a.grid, n_packets=a.packets)
    # the CPU baseline runs first, in forked workers, before anything touches the GPU
    cpu = cpu_baseline(wl, a.cpu_sample) if a.cpu_baseline else None

    import torch

    from paper_2507_11603_amd import thor

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    thor.lib()
    if a.calib_copy_mib:
        x = torch.empty(a.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    T = thor.Transport(0)
    T.load(wl["geom"])
    kw = dict(precision=a.precision, path=a.path, waves_per_cu=a.waves_per_cu, block=a.block,
              visits_per_turn=a.turn_visits, inline_peel=bool(a.inline_peel))
    tuned = None
    if a.autotune and a.path == "persistent" and not (a.waves_per_cu or a.block or a.turn_visits or a.inline_peel):
        from paper_2507_11603_amd import autotune
        tuned, _ = autotune.tune(T, wl, "shell%d" % a.grid, a.precision,
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
        kw.update(tuned)
    if a.warmup:
        run_steps(T, wl, a.packets, a.warmup, 10**12, **kw)
    dt, tot = run_steps(T, wl, a.packets, a.steps, 0, **kw)
    scat = tot["n_res"] + tot["n_dust"]
    value = scat / dt
    visits = tot["main_visits"] + tot["peel_visits"]
    kernel_s = tot["kernel_ms"] / 1e3
    achieved = BYTES_PER_VISIT * visits / a.steps / (kernel_s / a.steps) / 1e9
    out = {
        "metric": "photon scatterings/s on 1 MI355X (vs FP64 plain path)",
        "value": value,
        "unit": "scatterings/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "expanding shell r in [0.8, 1] on a %d^3 grid, N_HI 1e19, v_exp 200 km/s, "
                               "tau_d 0.5 (albedo 0.3), Gaussian source 20 km/s, dipole, +z peel cube "
                               "%dx%dx256" % (a.grid, a.grid, a.grid),
                   "packets_per_step": a.packets, "precision": a.precision, "path": a.path,
                   "waves_per_cu": kw["waves_per_cu"], "block": kw["block"],
                   "visits_per_turn": kw["visits_per_turn"], "autotuned": tuned is not None},
        "packets_per_s": tot["emitted"] / dt,
        "scatterings_per_packet": scat / max(tot["emitted"], 1),
        "cell_visits_per_s": visits / dt,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "launches": 1, "batches_per_launch": a.steps,
                     "kernel": "k_persistent<float,true>" if a.path == "persistent" else "k_plain",
                     "kernel_ms_per_step": tot["kernel_ms"] / a.steps, "upar_trials_per_scattering":
                         tot["upar_trials"] / max(tot["n_res"], 1),
                     "bytes_per_visit": BYTES_PER_VISIT, "visits_per_step": visits / a.steps},
    }
    tr = measured_traffic(a)
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes"]
        out["roofline"]["traffic_detail"] = tr
    if a.plain_steps:
        pdt, ptot = run_steps(T, wl, a.packets, a.plain_steps, 2 * 10**12, precision="fp64", path="plain")
        pval = (ptot["n_res"] + ptot["n_dust"]) / pdt
        out["plain_fp64"] = {"value": pval, "unit": "scatterings/s", "ms_per_step": pdt / a.plain_steps * 1e3,
                             "packets_per_s": ptot["emitted"] / pdt}
        out["speedup_vs_plain_fp64"] = value / pval
    T.close()
    if a.serving:
        out["serving"] = serving(a, kw)
    if a.web_grid:
        out["web"] = web_box(a, kw)
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
