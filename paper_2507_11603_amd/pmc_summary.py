"""Turn two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) over bench.py into
the per-batch HBM-side traffic record that bench.py reports as
`roofline.traffic`.

Both passes must profile the same bench.py command with `--calib-copy-mib M`:
its first dispatch is then a plain device copy of M MiB, which reads and writes
exactly M MiB, and the ratio of that to what each counter reports for it is the
counter's scale factor.  The timed persistent launch is the last dispatch of
`k_persistent`; its bytes are divided by the number of batches it ran.

The record carries a hash of the kernel sources; bench.py uses it only while
the hash matches the sources it was built from.

    python -m paper_2507_11603_amd.pmc_summary --fetch DIR_F --write DIR_W \
        --copy-mib 1024 --batches 3 --visits-per-batch V --out profiles/shell128_traffic.json
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/thor_lib.hip", "csrc/thor_engine.hpp", "csrc/thor_device.hpp"]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _per_dispatch(d: str):
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not path:
        raise FileNotFoundError("no counter_collection.csv under %s" % d)
    vals, names = collections.defaultdict(float), {}
    with open(path[0]) as f:
        for r in csv.DictReader(f):
            k = int(r["Dispatch_Id"])
            vals[k] += float(r["Counter_Value"])        # KiB, summed over XCD / instance rows
            names[k] = r["Kernel_Name"]
    return vals, names


def summarise(fetch_dir: str, write_dir: str, copy_mib: int, batches: int, visits_per_batch: float,
              kernel: str = "k_persistent") -> dict:
    out = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        vals, names = _per_dispatch(d)
        first = min(vals)
        if "copy" not in names[first].lower():
            raise ValueError("first dispatch %r is not the calibration copy" % names[first])
        scale = copy_mib * 1024.0 / vals[first]
        last = max(k for k in vals if kernel in names[k])
        out[key] = dict(scale=scale, calib_kib=vals[first], dispatch=last, raw_kib=vals[last],
                        bytes_per_batch=vals[last] * 1024.0 * scale / batches)
    alg = 20.0 * visits_per_batch
    return {"source_hash": source_hash(), "kernel": kernel, "batches_in_launch": batches,
            "fetch_bytes_per_batch": out["fetch"]["bytes_per_batch"],
            "write_bytes_per_batch": out["write"]["bytes_per_batch"],
            "algorithmic_bytes_per_batch": alg,
            "traffic_over_algorithmic": (out["fetch"]["bytes_per_batch"] + out["write"]["bytes_per_batch"]) / alg,
            "counters": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--batches", type=int, required=True)
    ap.add_argument("--visits-per-batch", type=float, required=True)
    ap.add_argument("--command", default="", help="the profiled command, stored with the record")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    rec = summarise(a.fetch, a.write, a.copy_mib, a.batches, a.visits_per_batch)
    rec["command"] = a.command
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
