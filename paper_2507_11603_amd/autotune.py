"""Autotuner for the persistent transport kernel.

Knobs: resident waves per CU (occupancy), workgroup size, and the number of
march segments a lane advances per turn (how often finished lanes are
refilled).  Each candidate transports the same short sample of the workload
(identical packets, so the work is identical); the lowest device time
without the tail kernel wins (the knobs shape the persistent kernel, while
the tail kernel's time follows the longest packet history of the sample).
Results are cached per (device, workload class, precision) in a JSON file.
"""
from __future__ import annotations

import json
import os

CACHE = os.environ.get("THOR_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "thor_autotune.json"))

DEFAULT_SPACE = dict(waves_per_cu=[4, 8, 12, 16], block=[256], visits_per_turn=[64, 256, 1024])


def _key(device_name: str, workload: str, precision: str) -> str:
    return "%s|%s|%s" % (device_name, workload, precision)


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


def tune(T, wl: dict, workload: str, precision: str = "mixed", sample: int = 200_000,
         batches: int = 2, space: dict | None = None, use_cache: bool = True, log=None):
    """Pick the fastest knob setting for `wl` on the context of Transport T.
    Returns (knobs dict, table of (knobs, seconds))."""
    import torch
    name = torch.cuda.get_device_name(T.device)
    key = _key(name, workload, precision)
    cache = load_cache()
    if use_cache and key in cache and cache[key].get("version") == 3:
        return cache[key]["best"], cache[key]["table"]
    space = space or DEFAULT_SPACE
    table = []
    for w in space["waves_per_cu"]:
        for b in space["block"]:
            for v in space["visits_per_turn"]:
                knobs = dict(waves_per_cu=w, block=b, visits_per_turn=v)
                T.reset()
                torch.cuda.synchronize()
                for i in range(batches):
                    T.emit(wl["src"], sample, 7 * 10**12 + i * sample)
                _, st = T.transport(wl["opts"], precision=precision, path="persistent", **knobs)
                # the knobs shape the persistent kernel; the tail kernel (the
                # few packets that run alone at the end, whose time is set by
                # the longest history in the sample) does not depend on them
                dt = (st["kernel_ms"] - st["tail_ms"]) / 1e3
                table.append((knobs, dt))
                if log:
                    log("autotune %s: %.1f ms without the tail kernel (%.1f ms)" % (knobs, dt * 1e3, st["tail_ms"]))
    best = min(table, key=lambda r: r[1])[0]
    cache[key] = dict(best=best, table=table, sample=sample, batches=batches, version=3)
    save_cache(cache)
    T.reset()
    return best, table
