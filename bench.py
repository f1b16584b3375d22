"""Benchmark of the Lyman-alpha packet-transport hot path on one MI355X.

Headline workload: the synthetic cosmic-web box on a 1024^3 grid (one GPU's
share of a large run).  One step = one thor_transport call over 1e8 packets
emitted in proportion to n_HI^2 with a thermal spectrum: march with the Voigt
cross-section in the gas frame, resonant scattering with core skipping at
x_crit = 3, dipole phase, peel-off to three axis observers (512^2 x 200
cubes), hand-off at the box faces.  Fields are built on the GPU (torch) and
loaded untimed; pencil records and allocations are made by the warm-up.

Prints one JSON line.  `value` is photon scatterings per second (resonant +
dust) of the persistent mixed-precision path over the timed steps; beside it:
the plain one-launch FP64 path on a sample of the same box, the roofline of
the dominant kernel, the 128^3 expanding shell, the serving stream, the
raytracing driver and the CPU oracle on a sample of the same box.
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
VALU_PEAK_IPS = 256 * 4 * 2.4e9 / 4    # wave64 VALU instructions/s: 256 CUs x 4 SIMDs, 1 per 4 cycles each
BYTES_PER_VISIT = 20.0         # (vx, vy, vz, n_HI, T) float32 per cell visit
METRIC = "photon scatterings/s on 1 MI355X (vs FP64 plain path); p50/p99 shell-request latency"
# knobs the autotuner searches on the web box (the others keep the library
# defaults; every candidate costs three runs of the steady-state sample)
WEB_SPACE = dict(park_lanes=[16, 32, 48], refill_64ths=[8, 16, 32], wide_lanes=[8, 16], presort=[0, 2, -1])
KERNEL_NAMES = {"transport": "k_persistent<float, true, true>", "tail": "k_tail<float, true, true>",
                "peel_pass": "k_peel_pass_f32"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1, help="timed thor_transport calls of --packets packets")
    ap.add_argument("--warmup", type=int, default=1, help="untimed calls of --warmup-packets packets first")
    ap.add_argument("--warmup-packets", type=int, default=1_000_000)
    ap.add_argument("--packets", type=int, default=100_000_000)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--fields", default="gpu",
                    help="gpu: torch on the device; cpu: numpy on the host; npy:DIR: saved numpy fields")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--waves-per-cu", type=int, default=8)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--turn-visits", type=int, default=0)
    ap.add_argument("--wide-lanes", type=int, default=0)
    ap.add_argument("--park-lanes", type=int, default=0)
    ap.add_argument("--refill-64ths", type=int, default=0)
    ap.add_argument("--seed-slots", type=int, default=0,
                    help="peel-seed buffer slots (48 B each; 0: library default, 2^28 to 2^30 by free memory)")
    ap.add_argument("--fuse-bins", type=int, default=0,
                    help="photon fusing of peel rays: sub-bins per cube frequency bin (0: off)")
    ap.add_argument("--seed-sort", type=int, default=0,
                    help="sort the peel seeds by pencil before each peel pass: 1 on, -1 off, 0 library default")
    ap.add_argument("--presort", type=int, default=0,
                    help="spatial presort of the queue: 1 on, -1 off, 0 the library default")
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick the launch knobs with the autotuner on a sample of the box first")
    ap.add_argument("--autotune-sample", type=int, default=4_000_000,
                    help="packets per autotuner run: enough for the steady state (a few dozen per lane), "
                         "so that the drain at the end of a launch does not decide")
    ap.add_argument("--plain-packets", type=int, default=20_000,
                    help="packets of the plain FP64 path on the same box (0: skip)")
    ap.add_argument("--shell", type=int, default=20, help="batches of 1e6 packets of the 128^3 shell (0: skip)")
    ap.add_argument("--shell-only", type=int, default=0, help="print only the shell record")
    ap.add_argument("--sphere", type=int, default=100_000,
                    help="packets of the meshless tau0 = 1e5 sphere, one persistent call (0: skip)")
    ap.add_argument("--sphere-only", type=int, default=0, help="print only the sphere record")
    ap.add_argument("--mg2", type=int, default=1_000_000,
                    help="packets per outflow velocity of the Mg II doublet sphere (0: skip)")
    ap.add_argument("--mg2-only", type=int, default=0, help="print only the Mg II record")
    ap.add_argument("--serving", type=int, default=300, help="measured requests of the serving stream (0: skip)")
    ap.add_argument("--serving-warmup", type=int, default=60)
    ap.add_argument("--serving-rate", type=float, default=200.0,
                    help="Poisson arrival rate (requests/s); one GPU sustains about 170/s")
    ap.add_argument("--serving-step-events", type=int, default=4096)
    ap.add_argument("--serving-only", type=int, default=0, help="print only the serving record")
    ap.add_argument("--rays", type=int, default=1, help="raytracing driver figures (0: skip)")
    ap.add_argument("--rays-only", type=int, default=0)
    ap.add_argument("--rays-grid", type=int, default=512)
    ap.add_argument("--rays-fields", default="cpu", choices=["cpu", "gpu"])
    ap.add_argument("--rays-reps", type=int, default=20)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--cpu-threads", type=int, default=16)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (PMC calibration)")
    ap.add_argument("--save-fields", default="", help="write the numpy fields to this directory and exit")
    return ap.parse_args()


# ------------------------------------------------------------------ helpers
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


def add_stats(tot, st):
    if tot is None:
        return dict(st)
    for k, v in st.items():
        if k == "max_events":
            tot[k] = max(tot[k], v)
        else:
            tot[k] = tot[k] + v
    return tot


def counter_record(name):
    """The committed counter record for workload `name`, or None when it is
    missing or the kernel sources have changed since it was taken."""
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_call(T, wl, n, first_id, **kw):
    """Queue n packets (ids first_id..) and transport them with one call."""
    import torch
    T.emit(wl["src"], n, first_id)
    code, st = T.transport(wl["opts"], **kw)
    torch.cuda.synchronize()
    assert st["emitted"] == n
    return st


# ------------------------------------------------------------------ web box
def web_fields(a):
    import numpy as np

    import workloads as W
    if a.fields == "gpu":
        return W.web_fields_torch(a.grid)
    if a.fields == "cpu":
        return W.web_fields(a.grid)
    if a.fields.startswith("npy:"):
        d = a.fields[4:]
        return tuple(np.load(os.path.join(d, "%s.npy" % k), mmap_mode="r")
                     for k in ("n_HI", "T", "vx", "vy", "vz"))
    raise ValueError("--fields gpu | cpu | npy:DIR")


def web_headline(a, kw):
    """Warm-up, then K timed calls of --packets packets on the web box.
    Returns the per-call totals, the wall time, the plain FP64 sample and
    (when the CPU baseline is asked for) host copies of the fields."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    f = web_fields(a)
    host = None
    if a.cpu_baseline:
        host = tuple(t.cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t) for t in f)
    wl = W.web(n_grid=a.grid, fields=f, n_packets=a.packets)
    T = thor.Transport(0)
    try:
        T.load(wl["geom"])
        for k in ("n_HI_field", "T_field", "vx", "vy", "vz"):
            wl["geom"][k] = None
        del f
        torch.cuda.empty_cache()
        if a.autotune:
            from paper_2507_11603_amd import autotune
            tuned, table = autotune.tune(T, wl, "web%d" % a.grid, a.precision, sample=a.autotune_sample,
                                         space=WEB_SPACE, log=lambda m: print(m, file=sys.stderr, flush=True))
            kw.update(tuned)
            kw["autotuned"] = {"sample": a.autotune_sample, "candidates": len(table)}
        knobs = {k: v for k, v in kw.items() if k != "autotuned"}
        for s in range(a.warmup):      # code loading, seed buffer, packet pool, pencil records
            run_call(T, wl, a.warmup_packets, 10**13 + s * a.warmup_packets, **knobs)
        T.reset()
        tot = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(a.steps):
            st = run_call(T, wl, a.packets, s * a.packets, **knobs)
            tot = add_stats(tot, st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        plain = None
        if a.plain_packets:
            t1 = time.perf_counter()
            pst = run_call(T, wl, a.plain_packets, 3 * 10**12, precision="fp64", path="plain")
            pdt = time.perf_counter() - t1
            plain = {"value": (pst["n_res"] + pst["n_dust"]) / pdt, "unit": "scatterings/s",
                     "packets": a.plain_packets, "seconds": pdt, "packets_per_s": a.plain_packets / pdt,
                     "scatterings_per_packet": (pst["n_res"] + pst["n_dust"]) / a.plain_packets,
                     "sample": "ids 3e12.. of the same box, one launch, one thread per packet, peel rays inline"}
    finally:
        T.close()
    return wl, tot, dt, plain, host


# What bounds each kernel of the grid path (counters on the 1024^3 box): the
# peel pass gathers pencil records (HBM), the transport and tail kernels issue
# VALU instructions on divergent histories (ALU).
KERNEL_BOUND = {"transport": "alu", "tail": "alu", "peel_pass": "hbm"}


def kernel_roofline(split, k):
    """Roofline block of kernel k: algorithmic bytes (20 B per cell visit) per
    launch over its average launch time against HBM; for an ALU-bound kernel
    the achieved figure is its VALU instruction rate, which needs a counter
    record (attach_counters) and stays None without one."""
    d = split[k]
    launches = max(d["launches"], 1)
    roof = {"bound": "hbm", "kernel": KERNEL_NAMES[k], "achieved": d["achieved_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["hbm_frac"], "traffic": None,
            "launches": d["launches"], "avg_launch_ms": d["ms"] / launches,
            "algorithmic_bytes_per_launch": BYTES_PER_VISIT * d["visits"] / launches,
            "bytes_per_visit": BYTES_PER_VISIT}
    if KERNEL_BOUND[k] == "alu":
        roof.update(bound="alu", achieved=None, peak=VALU_PEAK_IPS, unit="wave64 VALU instructions/s", frac=None,
                    hbm_achieved_GBps=d["achieved_GBps"], hbm_frac=d["hbm_frac"])
    return roof


def roofline_web(tot):
    split = kernel_split(tot)
    dom = max(split, key=lambda k: split[k]["ms"])
    return kernel_roofline(split, dom), split, dom


def attach_counters(roof, split, k, rec, packets):
    """From a counter record of the same workload (per packet there, scaled to
    this run): HBM bytes per launch of kernel k, and for an ALU-bound kernel
    its VALU instructions over its device time."""
    kname = {"transport": "k_persistent", "tail": "k_tail", "peel_pass": "k_peel_pass"}[k]
    kr = rec["kernels"].get(kname)
    if not kr:
        return
    scale = packets / max(rec["packets"], 1)
    launches = max(split[k]["launches"], 1)
    if "read_bytes_per_batch" in kr:
        roof["traffic"] = (kr["read_bytes_per_batch"] + kr["write_bytes_per_batch"]) * scale / launches
        roof["traffic_over_algorithmic"] = roof["traffic"] / roof["algorithmic_bytes_per_launch"]
    if roof["bound"] == "alu" and "valu_insts_per_batch" in kr and split[k]["ms"] > 0:
        ips = kr["valu_insts_per_batch"] * scale / (split[k]["ms"] / 1e3)
        roof.update(achieved=ips, frac=ips / VALU_PEAK_IPS, valu_busy_pct=kr.get("valu_busy_pct"),
                    valu_lane_util_pct=kr.get("valu_lane_util_pct"))
    roof["counters"] = rec["path"]


# ------------------------------------------------------------------ CPU oracle
def cpu_baseline(a, wl, host):
    """The oracle on a bounded sample of the same box (same fields, ids from
    0), on --cpu-threads host threads sharing one prepared medium, and on one
    thread; the sample is sized from a short calibration run."""
    import oracle
    oracle.build()
    geom = dict(wl["geom"])
    for k, v in zip(("n_HI_field", "T_field", "vx", "vy", "vz"), host):
        geom[k] = v
    threads = max(1, min(a.cpu_threads, os.cpu_count() or 1))
    cal = oracle.run_threaded(geom, wl["src"], wl["opts"], 0, 16 * threads, threads, reduce=False)
    per_packet = max(cal["transport_seconds"], 1e-3) / (16 * threads)
    n = int(max(8 * threads, min(2_000_000, a.cpu_seconds / per_packet)))
    r = oracle.run_threaded(geom, wl["src"], wl["opts"], 0, n, threads, reduce=False)
    scat = r["stats"]["n_res"] + r["stats"]["n_dust"]
    dt = r["transport_seconds"]
    n1 = int(max(4, min(200_000, a.cpu_seconds / 3.0 / (dt / n * threads))))
    r1 = oracle.run_threaded(geom, wl["src"], wl["opts"], 0, n1, 1, reduce=False)
    scat1 = r1["stats"]["n_res"] + r1["stats"]["n_dust"]
    return dict(value=scat / dt, unit="scatterings/s", cores=threads, kind="oracle",
                sample="packets 0..%d of the same %d^3 web box (seed 3), %d scatterings in %.1f s on %d "
                       "threads; the same box's first %d packets on 1 thread: %.3g scatterings/s"
                       % (n - 1, a.grid, scat, dt, threads, n1, scat1 / r1["transport_seconds"]),
                packets_per_s=n / dt, one_core_value=scat1 / r1["transport_seconds"],
                one_core_packets=n1, cpu_model=cpu_model(), host_cpus=os.cpu_count())


# ------------------------------------------------------------------ shell (secondary)
def shell_box(a):
    """Expanding shell on 128^3: a.shell batches of 1e6 packets in one call
    (one persistent launch); bound by VALU and by the longest history."""
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    wl = W.shell(n_grid=128, n_packets=1_000_000)
    T = thor.Transport(0)
    try:
        T.load(wl["geom"])
        kw = dict(precision="mixed", path="persistent", waves_per_cu=8)
        run_call(T, wl, 1_000_000, 10**12, **kw)
        T.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(a.shell):
            T.emit(wl["src"], 1_000_000, s * 1_000_000)
        _, st = T.transport(wl["opts"], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        T.close()
    split = kernel_split(st)
    dom = max(split, key=lambda k: split[k]["ms"])
    scat = st["n_res"] + st["n_dust"]
    out = {"workload": "expanding shell r in [0.8, 1] on a 128^3 grid, N_HI 1e19, v_exp 200 km/s, tau_d 0.5, "
                       "Gaussian source 20 km/s, dipole, +z cube 128x128x256",
           "batches": a.shell, "packets": st["emitted"], "seconds": dt, "scatterings_per_s": scat / dt,
           "packets_per_s": st["emitted"] / dt, "longest_history": st["max_events"],
           "kernels": split, "dominant": KERNEL_NAMES[dom]}
    rec = counter_record("shell128")
    roof = {"bound": "alu", "kernel": KERNEL_NAMES[dom], "achieved": None, "peak": VALU_PEAK_IPS,
            "unit": "wave64 VALU instructions/s", "frac": None}
    if rec is not None and dom in ("transport", "tail"):
        kr = rec["kernels"].get({"transport": "k_persistent", "tail": "k_tail"}[dom], {})
        if "valu_insts_per_batch" in kr and split[dom]["ms"] > 0:
            ips = kr["valu_insts_per_batch"] * a.shell / (split[dom]["ms"] / 1e3)
            roof.update(achieved=ips, frac=ips / VALU_PEAK_IPS, counters=rec["path"])
    out["roofline"] = roof
    return out


def serving(a):
    """Open-loop stream of shell-model requests through the continuous-batching
    server: p50/p99 latency (completion - arrival) and sustained throughput."""
    import numpy as np

    import workloads as W
    from paper_2507_11603_amd import serve
    stream = W.request_stream(a.serving + a.serving_warmup, rate_hz=a.serving_rate)
    srv = serve.ShellServer(precision=a.precision, step_events=a.serving_step_events)
    try:
            r = srv.run_stream(stream, warmup=a.serving_warmup, progress_s=20.0)
    finally:
        srv.close()
    pk = sum(q["n_packets"] for q in stream)
    span = stream[-1]["t_arrival"] - stream[0]["t_arrival"]
    return {"requests": a.serving, "warmup_requests": a.serving_warmup, "rate_hz": a.serving_rate,
            "p50_ms": r["p50_s"] * 1e3, "p90_ms": float(np.percentile(r["latency_s"], 90)) * 1e3,
            "p99_ms": r["p99_s"] * 1e3, "sustained_requests_per_s": len(stream) / r["wall_s"],
            "offered_packets_per_s": pk / span, "sustained_packets_per_s": pk / r["wall_s"],
            "sustained_scatterings_per_s": r["scatterings"] / r["wall_s"], "wall_s": r["wall_s"],
            "steps": r["steps"], "step_events": a.serving_step_events, "budget_deferrals": r["deferrals"],
            "graph_steps": True}


def sphere_box(a):
    """The meshless static sphere (tau0 = 1e5, T = 1e4 K, line-centre point
    source, isotropic phase, no dust, no core skipping): a.sphere packets in
    one persistent call.  No field memory: bound by VALU issue; the roofline
    takes the VALU instructions per packet from the sphere's counter record."""
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    wl = W.sphere(tau0=1e5, n_packets=a.sphere)
    T = thor.Transport(0)
    try:
        T.load(wl["geom"])
        kw = dict(precision="mixed", path="persistent", waves_per_cu=8)
        run_call(T, wl, max(1, a.sphere // 10), 10**12, **kw)     # warm-up
        T.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.emit(wl["src"], a.sphere, 0)
        _, st = T.transport(wl["opts"], **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    finally:
        T.close()
    split = kernel_split(st)
    scat = st["n_res"] + st["n_dust"]
    out = {"workload": "static sphere tau0 = 1e5, T = 1e4 K, x = 0 point source, isotropic, no dust",
           "packets": st["emitted"], "seconds": dt, "scatterings_per_s": scat / dt,
           "scatterings_per_packet": scat / max(st["emitted"], 1), "kernel_ms": st["kernel_ms"],
           "upar_trials_per_scattering": st["upar_trials"] / max(st["n_res"], 1),
           "longest_history": st["max_events"], "kernels": split}
    roof = {"bound": "alu", "kernel": "k_persistent<float, false, false>", "achieved": None,
            "peak": VALU_PEAK_IPS, "unit": "wave64 VALU instructions/s", "frac": None}
    rec = counter_record("sphere")
    if rec is not None:
        kr = rec["kernels"].get("k_persistent", {})
        if "valu_insts_per_batch" in kr and split["transport"]["ms"] > 0:
            ips = kr["valu_insts_per_batch"] / max(rec["packets"], 1) * st["emitted"] / (split["transport"]["ms"] / 1e3)
            roof.update(achieved=ips, frac=ips / VALU_PEAK_IPS, counters=rec["path"],
                        valu_busy_pct=kr.get("valu_busy_pct"), valu_lane_util_pct=kr.get("valu_lane_util_pct"))
    out["roofline"] = roof
    return out


def mg2_box(a):
    """Section 4's doublet test: the Mg II sphere (column 10^14.5 cm^-2,
    T = 1e4 K) with the linear outflow v = v_max r/R for v_max = 100, 200,
    500, 1000 km/s, lit by a flat continuum over -1500..1000 km/s around the
    k line; a.mg2 packets per velocity, mixed precision, one persistent call
    each.  Reports the throughput and the share of the escaping flux blueward
    of the doublet's midpoint, F_blue / F_tot."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2507_11603_amd import thor
    out = {"workload": "Mg II h+k sphere, N = 10^14.5 cm^-2, T = 1e4 K, linear outflow, flat continuum "
                       "-1500..1000 km/s, dipole (k) / isotropic (h)", "packets": a.mg2, "runs": []}
    c_h = -767.6e5
    for v in (100.0, 200.0, 500.0, 1000.0):
        wl = W.mg2_sphere(v_max_kms=v, n_packets=a.mg2)
        T = thor.Transport(0)
        try:
            T.load(wl["geom"])
            kw = dict(precision="mixed", path="persistent", waves_per_cu=8, presort=a.presort)
            run_call(T, wl, max(1, a.mg2 // 10), 10**12, **kw)
            T.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            T.emit(wl["src"], a.mg2, 0)
            _, st = T.transport(wl["opts"], **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            spec = T.spectrum()
        finally:
            T.close()
        sp = wl["opts"]["spectrum"]
        centres = sp["lo"] + (np.arange(sp["nb"]) + 0.5) * (sp["hi"] - sp["lo"]) / sp["nb"]
        out["runs"].append({"v_max_kms": v, "seconds": dt, "packets_per_s": st["emitted"] / dt,
                            "scatterings_per_s": (st["n_res"] + st["n_dust"]) / dt,
                            "scatterings_per_packet": st["n_res"] / max(st["emitted"], 1),
                            "segments_per_s": st["main_visits"] / (st["kernel_ms"] / 1e3),
                            "blue_fraction": float(spec[centres > 0.5 * c_h].sum() / spec.sum()),
                            "spectrum_50_bins": [int(x) for x in spec.reshape(50, -1).sum(axis=1)]})
    return out


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


def save_fields(a):
    """The web box's fields (--fields gpu or cpu) as numpy files in a
    directory, for the counter runs, which load them (--fields npy:DIR)
    instead of generating them under the profiler once per pass."""
    import numpy as np

    os.makedirs(a.save_fields, exist_ok=True)
    for k, v in zip(("n_HI", "T", "vx", "vy", "vz"), web_fields(a)):
        v = v.cpu().numpy() if hasattr(v, "cpu") else np.asarray(v)
        np.save(os.path.join(a.save_fields, "%s.npy" % k), v)
        print("saved %s" % k, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.save_fields:
        save_fields(a)
        return
    import torch

    from paper_2507_11603_amd import thor
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    thor.lib()
    calib_copy(a)
    if a.rays_only:
        print(json.dumps({"rays": rays_box(a, device_fields=a.rays_fields == "gpu")}), flush=True)
        return
    if a.serving_only:
        print(json.dumps({"serving": serving(a)}), flush=True)
        return
    if a.sphere_only:
        print(json.dumps({"sphere": sphere_box(a)}), flush=True)
        return
    if a.shell_only:
        print(json.dumps({"shell": shell_box(a)}), flush=True)
        return
    if a.mg2_only:
        print(json.dumps({"mg2": mg2_box(a)}), flush=True)
        return
    kw = dict(precision=a.precision, path="persistent", waves_per_cu=a.waves_per_cu, block=a.block or 256,
              visits_per_turn=a.turn_visits or 256, wide_lanes=a.wide_lanes or 8, park_lanes=a.park_lanes or 32,
              refill_64ths=a.refill_64ths or 16, presort=a.presort, seed_sort=a.seed_sort,
              fuse_bins=a.fuse_bins, seed_slots=a.seed_slots)
    wl, tot, dt, plain, host = web_headline(a, kw)
    print("[bench] web %d^3: %d packets in %.2f s" % (a.grid, tot["emitted"], dt), file=sys.stderr, flush=True)
    scat = tot["n_res"] + tot["n_dust"]
    value = scat / dt
    roof, split, dom = roofline_web(tot)
    gather = kernel_roofline(split, "peel_pass")
    rec = counter_record("web%d" % a.grid) if a.precision == "mixed" else None
    if rec is not None and rec.get("fields") == a.fields:
        attach_counters(roof, split, dom, rec, a.packets * a.steps)
        attach_counters(gather, split, "peel_pass", rec, a.packets * a.steps)
    visits = tot["main_visits"] + tot["peel_visits"]
    ks = tot["kernel_ms"] / 1e3
    path_gbs = BYTES_PER_VISIT * visits / ks / 1e9
    out = {
        "metric": METRIC,
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
        "config": {"workload": "cosmic-web box %d^3 (L = 17.22 pMpc, log n_HI Gaussian random field P(k) ~ k^-2.5, "
                               "sigma_ln 2, mean 1e-5 cm^-3, T = 1e4 K (n/mean)^0.5, velocity fields 100 km/s), "
                               "%d packets per step emitted ~ n_HI^2, thermal spectrum, x_crit 3, dipole, three "
                               "axis observers 512x512x200, face exits handed off" % (a.grid, a.packets),
                   "packets_per_step": a.packets, "warmup_packets": a.warmup_packets, "fields": a.fields,
                   "precision": a.precision, "path": "persistent",
                   "knobs": {k: kw[k] for k in ("waves_per_cu", "block", "visits_per_turn", "wide_lanes",
                                                "park_lanes", "refill_64ths", "presort", "seed_sort",
                                                "fuse_bins", "seed_slots")},
                   "autotuned": kw.get("autotuned")},
        "packets_per_s": tot["emitted"] / dt,
        "scatterings_per_packet": scat / max(tot["emitted"], 1),
        "cell_visits_per_s": visits / ks,
        "path_hbm": {"achieved": path_gbs, "frac": path_gbs / HBM_PEAK_GBS, "kernel_ms": tot["kernel_ms"],
                     "main_visits": tot["main_visits"], "peel_visits": tot["peel_visits"]},
        "roofline": roof,
        # the peel pass's HBM-gather figure, whichever kernel dominates
        "hbm_gather": gather,
        "kernels": split,
        "passes": tot["passes"],
        "presort_ms": tot.get("presort_ms", 0.0),
        "seedsort_ms": tot.get("seedsort_ms", 0.0),
        "peel_fused": tot.get("peel_fused", 0),
        "longest_history": tot["max_events"],
    }
    if plain:
        out["plain_fp64"] = plain
        out["speedup_vs_plain_fp64"] = value / plain["value"]
    del wl["geom"]
    if a.shell:
        out["shell"] = shell_box(a)
    if a.sphere:
        out["sphere"] = sphere_box(a)
    if a.mg2:
        out["mg2"] = mg2_box(a)
    if a.serving:
        out["serving"] = serving(a)
    if a.rays:
        r = rays_box(a, device_fields=True)
        out["rays"] = {"workload": r["workload"] + " (device-built fields)",
                       "projection_GBps": {k: v["achieved_GBps"] for k, v in r["projection"].items()},
                       "projection_hbm_frac": {k: v["hbm_frac"] for k, v in r["projection"].items()},
                       "forest_ms": {k: v["ms"] for k, v in r["forest"].items()},
                       "forest_voigt_evals_per_s": {k: v["voigt_evals_per_s"] for k, v in r["forest"].items()},
                       "forest_rays": r["forest"]["fp64"]["rays"]}
    if a.cpu_baseline and host is not None:
        import workloads as W
        out["cpu_baseline"] = cpu_baseline(a, W.web(n_grid=a.grid, fields=host, n_packets=a.packets), host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
