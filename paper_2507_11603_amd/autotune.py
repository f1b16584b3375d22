"""Autotuner for the persistent transport kernel (the batching form).

Knobs (thor_transport_opts): resident waves per CU and workgroup size (the
packet slots of the launch: lanes x one packet each), park_lanes (how many
lanes wait at their interaction sites before they interact together),
refill_64ths (the share of a turn's lanes that must have finished before the
wave ends the turn and refills them), wide_lanes (the live-lane count at
which a drained wave hands its packets to the tail kernel), visits_per_turn
and presort (the order in which queued packets are taken: the library
default, by emitted frequency, or as queued).

Every candidate transports the same sample of the workload (the same photon
ids, hence the same histories and the same work); its score is the median
over `repeats` runs of the call's total device time (transport, tail and
peel-pass kernels).  The search is coordinate-wise: starting from the
library defaults, each knob in turn takes the value with the lowest score
while the others stay fixed.  Results are cached per (device, workload,
precision, sample) in a JSON file.
"""
from __future__ import annotations

import json
import os
import statistics

CACHE = os.environ.get("THOR_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "thor_autotune.json"))

DEFAULTS = dict(waves_per_cu=8, block=256, park_lanes=32, refill_64ths=16, wide_lanes=8, visits_per_turn=256,
                presort=0)
SPACE = dict(park_lanes=[-1, 16, 24, 32, 40], refill_64ths=[8, 16, 32, 64], waves_per_cu=[4, 8],
             block=[64, 128, 256], wide_lanes=[4, 8, 16], visits_per_turn=[64, 256, 1024], presort=[0, 2, -1])
VERSION = 5


def _key(device_name: str, workload: str, precision: str, sample: int) -> str:
    return "%s|%s|%s|%d" % (device_name, workload, precision, sample)


def load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def score(T, wl: dict, precision: str, sample: int, knobs: dict, repeats: int, first_id: int) -> float:
    """Median total device time (ms) of `repeats` calls over the same sample."""
    times = []
    for _ in range(repeats):
        T.reset()
        T.emit(wl["src"], sample, first_id)
        _, st = T.transport(wl["opts"], precision=precision, path="persistent", **knobs)
        times.append(st["kernel_ms"])
    return statistics.median(times)


def tune(T, wl: dict, workload: str, precision: str = "mixed", sample: int = 500_000, repeats: int = 3,
         space: dict | None = None, use_cache: bool = True, log=None):
    """Pick knob values for `wl` on the context of Transport T (its medium
    loaded).  Returns (knobs, table of (knobs, median ms))."""
    import torch
    name = torch.cuda.get_device_name(T.device)
    key = _key(name, workload, precision, sample)
    cache = load_cache()
    if use_cache and key in cache and cache[key].get("version") == VERSION:
        return cache[key]["best"], cache[key]["table"]
    space = space or SPACE
    first_id = 7 * 10**12
    best = dict(DEFAULTS)
    seen = {}

    def measure(k):
        t = tuple(sorted(k.items()))
        if t not in seen:
            seen[t] = score(T, wl, precision, sample, k, repeats, first_id)
            if log:
                log("autotune %s: %.1f ms" % (k, seen[t]))
        return seen[t]

    score(T, wl, precision, sample, best, 1, first_id)      # warm-up: allocations, pencil records
    for knob, values in space.items():
        cands = []
        for v in values:
            k = dict(best, **{knob: v})
            cands.append((measure(k), v))
        best[knob] = min(cands)[1]
    table = [(dict(t), ms) for t, ms in seen.items()]
    cache[key] = dict(best=best, table=table, sample=sample, repeats=repeats, version=VERSION)
    save_cache(cache)
    T.reset()
    return best, table
