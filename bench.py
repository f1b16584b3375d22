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
    ap.add_argument("--steps", type=int, default=100,
                    help="batches of 1e6 packets transported by one call (one persistent launch)")
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
    ap.add_argument("--cpu-sample", type=int, default=8_000_000,
                    help="packets of the oracle sample (ids 0..n-1; about 15 s on 16 host cores)")
    ap.add_argument("--autotune", type=int, default=1, help="pick launch knobs with the autotuner")
    ap.add_argument("--serving", type=int, default=300, help="requests of the serving stream (0: skip)")
    ap.add_argument("--serving-warmup", type=int, default=60)
    ap.add_argument("--serving-rate", type=float, default=200.0)
    ap.add_argument("--serving-step-events", type=int, default=4096,
                    help="interactions per lane per serving step (longer steps: fewer launches and host syncs)")
    ap.add_argument("--web-grid", type=int, default=0,
                    help="also measure the cosmic-web box at this grid size (fields generated on the GPU)")
    ap.add_argument("--web-packets", type=int, default=100_000)
    ap.add_argument("--web-fields", default="gpu", choices=["gpu", "cpu"],
                    help="make the web fields with torch on the GPU or with numpy on the host")
    ap.add_argument("--web-only", type=int, default=0,
                    help="measure only the cosmic-web box and print its record (for counter runs)")
    ap.add_argument("--web-warmup", type=int, default=1, help="untimed web run of a tenth of the packets first")
    ap.add_argument("--rays-only", type=int, default=0,
                    help="time only the raytracing driver (projections and forest spectra) on the web box")
    ap.add_argument("--rays", type=int, default=1,
                    help="add the raytracing driver's figures (device-built fields) to the bench line")
    ap.add_argument("--rays-grid", type=int, default=512)
    ap.add_argument("--rays-fields", default="cpu", choices=["cpu", "gpu"],
                    help="--rays-only fields: numpy-built (as the parity tests) or device-built")
    ap.add_argument("--rays-reps", type=int, default=20, help="timed launches per raytracing kernel")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (PMC calibration)")
    return ap.parse_args()


def kernel_split(st):
    """Device time and algorithmic cell visits of the kernels of a call.
    Persistent path: the persistent kernel marches main flights and, on the
    peel-seed path, the first segment of every peel ray (one visit per ray);
    the tail kernel does the same for the packets handed off at the end of
    the launch; the peel pass marches the rest of the rays.  Plain path or
    inline peel: the transport kernel does everything."""
    seeded = st["peel_ms"] > 0.0
    tail_ms = st.get("tail_ms", 0.0)
    tl_visits = st.get("tail_main_visits", 0) + st.get("tail_peel_visits", 0)
    tr_visits = st["main_visits"] + (st["peel_contrib"] if seeded else st["peel_visits"]) - tl_visits
    pp_visits = st["peel_visits"] - st["peel_contrib"] if seeded else 0
    out = {}
    for name, ms, v in (("transport", st["transport_ms"] - tail_ms, tr_visits), ("tail", tail_ms, tl_visits),
                        ("peel_pass", st["peel_ms"], pp_visits)):
        if name == "tail" and ms <= 0.0:
            continue
        ach = BYTES_PER_VISIT * v / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        out[name] = {"ms": ms, "visits": v, "launches": int(st["passes"]) if (ms > 0 or name == "transport") else 0,
                     "achieved_GBps": ach, "hbm_frac": ach / HBM_PEAK_GBS}
    if "tail" in out:
        out["tail"]["events"] = st["tail_events"]
    return out


def counter_record(name):
    """The committed counter record for workload `name` (two HBM byte passes
    calibrated on a plain copy, one VALU pass), or None when it is missing or
    the kernel sources have changed since it was taken."""
    from paper_2507_11603_amd import pmc_summary
    path = os.path.join(ROOT, "profiles", "%s_counters.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != pmc_summary.source_hash():
        return None
    rec["path"] = os.path.relpath(path, ROOT)
    return rec


def attach_counters(roof, split, dom, rec, batches):
    """HBM traffic per launch of the dominant kernel and VALU activity of both
    kernels from a counter record (per batch there, scaled to this run)."""
    kname = {"transport": "k_persistent", "tail": "k_tail", "peel_pass": "k_peel_pass"}[dom]
    kr = rec["kernels"].get(kname)
    if kr and "read_bytes_per_batch" in kr and "write_bytes_per_batch" in kr:
        launches = max(split[dom]["launches"], 1)
        per_batch = kr["read_bytes_per_batch"] + kr["write_bytes_per_batch"]
        roof["traffic"] = per_batch * batches / launches
        roof["traffic_over_algorithmic"] = roof["traffic"] / (BYTES_PER_VISIT * split[dom]["visits"] / launches)
    roof["counters"] = {"record": rec["path"], "kernels": rec["kernels"],
                        "read_check": rec.get("read_check"), "write_scale": rec.get("write_scale")}


def calib_copy(a):
    """A plain device copy of --calib-copy-mib MiB (reads and writes that many
    bytes): the reference dispatch that scales the HBM byte counters."""
    if not a.calib_copy_mib:
        return
    import torch
    x = torch.empty(a.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y


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
    srv = serve.ShellServer(precision=a.precision, step_events=a.serving_step_events,
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
            "steps": r["steps"], "step_events": a.serving_step_events, "budget_deferrals": r["deferrals"],
            "graph_steps": True}


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
        if a.web_warmup:
            run_steps(T, wl, a.web_packets // 10, 1, 10**13, **wkw)       # warm-up (caches, allocations)
        dt, st = run_steps(T, wl, a.web_packets, 1, 0, **wkw)
    finally:
        T.close()
    visits = st["main_visits"] + st["peel_visits"]
    ks = st["kernel_ms"] / 1e3
    ach = BYTES_PER_VISIT * visits / ks / 1e9
    split = kernel_split(st)
    dom = max(split, key=lambda k: split[k]["ms"])
    roof = {"bound": "hbm", "kernel": dom, "achieved": split[dom]["achieved_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": split[dom]["hbm_frac"], "traffic": None}
    rec = counter_record("web%d" % a.web_grid) if (a.path == "persistent" and a.precision == "mixed") else None
    # the counter record was taken on the numpy-built fields (no torch kernels under the profiler)
    if rec is not None and rec.get("packets") == a.web_packets and a.web_fields == "cpu":
        attach_counters(roof, split, dom, rec, 1)
    return {"grid": a.web_grid, "packets": a.web_packets, "seconds": dt, "kernel_ms": st["kernel_ms"],
            "scatterings_per_s": (st["n_res"] + st["n_dust"]) / dt, "packets_per_s": st["emitted"] / dt,
            "main_visits": st["main_visits"], "peel_visits": st["peel_visits"],
            "cell_visits_per_s": visits / ks, "passes": st["passes"],
            "path_hbm": {"achieved": ach, "frac": ach / HBM_PEAK_GBS},
            "kernels": split,
            "roofline": roof}


def rays_box(a, device_fields=False):
    """Raytracing driver on the forest workload (web box at z = 2): column-
    density projections along each axis (HBM-bound: 4 B read per cell) and
    the absorption spectra of one tomography plane, FP64 and mixed (bound by
    the Voigt evaluations: rays x cells x sub-steps x bins)."""
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    wl = W.forest(a.rays_grid, device="cuda" if device_fields else None)
    o = wl["opts"]
    n, T, v = (f if device_fields else torch.from_numpy(f).cuda() for f in wl["fields"])
    cells = n.numel()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()                                           # warm-up launch
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    out = {"workload": "forest%d" % a.rays_grid, "cells": cells, "projection": {}, "forest": {}}
    for axis, name in enumerate("xyz"):
        img = thor.ray_project(n, None, axis, o["ds"])
        ms = timed(lambda: thor.ray_project(n, None, axis, o["ds"], out=img), a.rays_reps)
        nbytes = 4 * cells + 2 * 8 * img[0].numel()
        gbs = nbytes / (ms / 1e3) / 1e9
        out["projection"][name] = {"ms": ms, "bytes": nbytes, "achieved_GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    i0, ni, j0, nj = o["rays"]
    evals = ni * nj * a.rays_grid * o["n_sub"] * o["nb"]
    for prec in ("fp64", "mixed"):
        tau = thor.ray_forest(n, T, v, o["axis"], o["ds"], o["hubble"], o["n_sub"], o["rays"], o["nb"],
                              o["u_lo"], o["u_hi"], prec)
        ms = timed(lambda: thor.ray_forest(n, T, v, o["axis"], o["ds"], o["hubble"], o["n_sub"], o["rays"],
                                           o["nb"], o["u_lo"], o["u_hi"], prec, out=tau),
                   max(1, a.rays_reps // 4))
        out["forest"][prec] = {"ms": ms, "rays": ni * nj, "voigt_evals": evals,
                               "voigt_evals_per_s": evals / (ms / 1e3),
                               "median_tau": float(tau.median().item())}
    z = out["projection"]["z"]
    out["roofline"] = {"bound": "hbm", "kernel": "k_project_cols (axis z)", "achieved": z["achieved_GBps"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": z["hbm_frac"], "traffic": None}
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.rays_only:
        import torch

        from paper_2507_11603_amd import thor
        if not torch.cuda.is_available():
            print("no HIP device", file=sys.stderr)
            sys.exit(1)
        thor.lib()
        calib_copy(a)
        print(json.dumps({"rays": rays_box(a, device_fields=a.rays_fields == "gpu")}), flush=True)
        return
    if a.web_only:
        import torch

        from paper_2507_11603_amd import thor
        if not torch.cuda.is_available():
            print("no HIP device", file=sys.stderr)
            sys.exit(1)
        thor.lib()
        calib_copy(a)
        kw = dict(precision=a.precision, path=a.path, waves_per_cu=a.waves_per_cu, block=a.block,
                  inline_peel=bool(a.inline_peel))
        print(json.dumps({"web": web_box(a, kw)}), flush=True)
        return
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
    calib_copy(a)
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
    split = kernel_split(tot)
    dom = max(split, key=lambda k: split[k]["ms"])
    achieved = split[dom]["achieved_GBps"]
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
                     "kernel": ({"transport": "k_persistent<float,true,true>", "tail": "k_tail<float,true,true>",
                                 "peel_pass": "k_peel_pass_f32"}[dom] if a.path == "persistent" else "k_plain"),
                     "launches": split[dom]["launches"], "batches_per_launch": a.steps / max(split[dom]["launches"], 1),
                     "kernel_ms": split[dom]["ms"], "visits": split[dom]["visits"],
                     "bytes_per_visit": BYTES_PER_VISIT,
                     "upar_trials_per_scattering": tot["upar_trials"] / max(tot["n_res"], 1)},
        "kernels": split,
        # the step ends when its longest packet history does: a few packets per
        # million scatter 1e4-1e6 times near line centre, and the last of them
        # run alone, one lane's serial chain of interactions each
        "longest_history": {"events": tot["max_events"],
                            "us_per_event_if_alone_for_the_step": dt * 1e6 / max(tot["max_events"], 1),
                            "tail_kernel_ms": tot.get("tail_ms", 0.0), "tail_events": tot.get("tail_events", 0)},
    }
    rec = counter_record("shell%d" % a.grid) if (a.path == "persistent" and a.precision == "mixed") else None
    if rec is not None:
        attach_counters(out["roofline"], split, dom, rec, a.steps)
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
    if a.rays:
        r = rays_box(a, device_fields=True)
        out["rays"] = {"workload": r["workload"] + " (device-built fields)",
                       "projection_GBps": {k: v["achieved_GBps"] for k, v in r["projection"].items()},
                       "projection_hbm_frac": {k: v["hbm_frac"] for k, v in r["projection"].items()},
                       "forest_ms": {k: v["ms"] for k, v in r["forest"].items()},
                       "forest_voigt_evals_per_s": {k: v["voigt_evals_per_s"] for k, v in r["forest"].items()},
                       "forest_rays": r["forest"]["fp64"]["rays"]}
    if cpu:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
