"""Turn rocprofv3 counter passes over one bench.py command into the record
bench.py reports beside its roofline: bytes the L2 caches read from and
write to the memory fabric, and VALU activity (VALUBusy, VALUUtilization,
SQ_INSTS_VALU), per kernel and per batch.

Reads come from FETCH_SIZE and writes from WRITE_SIZE (KiB per dispatch),
each scaled by what it reports for a plain device copy of known size: the
passes must profile the same command, run with `--warmup 0` (so every
dispatch of a kernel belongs to the timed call) and `--calib-copy-mib M`, so
that the first dispatch copies exactly M MiB (reads and writes M MiB).  The
derived FETCH_SIZE counts a 128-byte request as 64 bytes, so its copy scale
is about 2; a kernel whose requests are smaller than the copy's is then
over-counted by up to that factor.  An optional pass over the L2 read
requests by size (TCC_EA0_RDREQ_32B, _64B, _128B; bytes = 32 n32 + 64 n64 +
128 n128) gives the reads without that assumption, kept beside them.

The record carries a hash of the kernel sources; bench.py uses it only while
the hash matches the sources it was built from.

    python -m paper_2507_11603_amd.pmc_summary --fetch DIR --write DIR [--reads DIR] \\
        [--valu DIR] [--hits DIR] --copy-mib 1024 --batches 1 --packets N --out RECORD.json
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
KERNELS = ("k_persistent", "k_tail", "k_peel_pass")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(d: str):
    path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not path:
        raise FileNotFoundError("no counter_collection.csv under %s" % d)
    with open(path[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter):
    vals, names = collections.defaultdict(float), {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        vals[k] += float(r["Counter_Value"])        # summed over XCD / instance rows
        names[k] = r["Kernel_Name"]
    return vals, names


def _durations(rows):
    return {int(r["Dispatch_Id"]): int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows}


def _pick(ds, last_only):
    """Dispatches of one kernel: all of them, or only the last (the timed call
    of a command whose warm-up call comes first)."""
    return [max(ds)] if (last_only and ds) else ds


def _scaled_kib(d: str, counter: str, copy_mib: int, batches: int, rec: dict, key: str, scale_key: str,
                last_only: bool = False):
    """Per-batch bytes of `counter` (KiB per dispatch) for each kernel, scaled
    by the calibration copy (the first dispatch)."""
    vals, names = _per_dispatch(_rows(d), counter)
    first = min(vals)
    if "copy" not in names[first].lower():
        raise ValueError("first dispatch %r is not the calibration copy" % names[first])
    scale = copy_mib * 1024.0 / vals[first]
    rec[scale_key] = scale
    for kname in KERNELS:
        ds = _pick([k for k in vals if kname in names[k]], last_only)
        if ds:
            kr = rec["kernels"].setdefault(kname, {})
            kr["launches"] = len(ds)
            kr[key] = sum(vals[k] for k in ds) * 1024.0 * scale / batches


def summarise(fetch_dir: str | None, write_dir: str, valu_dir: str | None, copy_mib: int, batches: int,
              packets: int = 0, hits_dir: str | None = None, reads_dir: str | None = None,
              last_only: bool = False) -> dict:
    rec = {"source_hash": source_hash(), "batches": batches, "packets": packets, "kernels": {}}
    if last_only:
        rec["dispatches"] = "last of each kernel"
    if fetch_dir:
        _scaled_kib(fetch_dir, "FETCH_SIZE", copy_mib, batches, rec, "read_bytes_per_batch", "fetch_scale",
                    last_only)
    if reads_dir:
        # reads from the request counts by size
        rows = _rows(reads_dir)
        per = {sz: _per_dispatch(rows, "TCC_EA0_RDREQ_%dB" % sz) for sz in (32, 64, 128)}
        names = per[128][1]
        rbytes = collections.defaultdict(float)
        for sz, (vals, _) in per.items():
            for k, v in vals.items():
                rbytes[k] += sz * v
        first = min(rbytes)
        if "copy" not in names[first].lower():
            raise ValueError("first dispatch %r is not the calibration copy" % names[first])
        rec["read_check"] = rbytes[first] / (copy_mib * 2.0 ** 20)     # 1.0: the copy reads what it copies
        key = "read_req_bytes_per_batch" if fetch_dir else "read_bytes_per_batch"
        for kname in KERNELS:
            ds = _pick([k for k in rbytes if kname in names[k]], last_only)
            if ds:
                kr = rec["kernels"].setdefault(kname, {})
                kr["launches"] = len(ds)
                kr[key] = sum(rbytes[k] for k in ds) / batches
    _scaled_kib(write_dir, "WRITE_SIZE", copy_mib, batches, rec, "write_bytes_per_batch", "write_scale", last_only)
    if hits_dir:
        rows = _rows(hits_dir)
        for kname in KERNELS:
            kr_rows = [r for r in rows if kname in r["Kernel_Name"]]
            hit, _ = _per_dispatch(kr_rows, "TCC_HIT")
            miss, _ = _per_dispatch(kr_rows, "TCC_MISS")
            h, m = sum(hit.values()), sum(miss.values())
            if h + m > 0:
                rec["kernels"].setdefault(kname, {})["l2_hit_pct"] = 100.0 * h / (h + m)
    if valu_dir:
        rows = _rows(valu_dir)
        for kname in KERNELS:
            kr_rows = [r for r in rows if kname in r["Kernel_Name"]]
            busy, _ = _per_dispatch(kr_rows, "VALUBusy")
            util, _ = _per_dispatch(kr_rows, "VALUUtilization")
            insts, _ = _per_dispatch(kr_rows, "SQ_INSTS_VALU")
            if last_only and insts:
                insts = {max(insts): insts[max(insts)]}
            if not insts:
                continue
            dur = _durations(kr_rows)
            kr = rec["kernels"].setdefault(kname, {})
            # per-dispatch percentages: busy (a share of time) weighted by
            # duration, lane utilisation (a share per instruction) by instructions
            t_tot = sum(dur[k] for k in insts)
            i_tot = sum(insts.values())
            kr["valu_busy_pct"] = sum(busy.get(k, 0.0) * dur[k] for k in insts) / t_tot if t_tot else 0.0
            kr["valu_lane_util_pct"] = sum(util.get(k, 0.0) * insts[k] for k in insts) / i_tot if i_tot else 0.0
            kr["valu_insts_per_batch"] = i_tot / batches
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", default=None, help="pass with FETCH_SIZE")
    ap.add_argument("--reads", default=None, help="pass with TCC_EA0_RDREQ_32B/_64B/_128B")
    ap.add_argument("--write", required=True, help="pass with WRITE_SIZE")
    ap.add_argument("--valu", default=None, help="pass with VALUBusy VALUUtilization SQ_INSTS_VALU")
    ap.add_argument("--hits", default=None, help="pass with TCC_HIT TCC_MISS")
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--batches", type=int, required=True)
    ap.add_argument("--packets", type=int, default=0, help="packets per batch")
    ap.add_argument("--command", default="", help="the profiled command, stored with the record")
    ap.add_argument("--fields", default="", help="bench.py --fields of the profiled command")
    ap.add_argument("--last-only", action="store_true",
                    help="count only the last dispatch of each kernel (the timed call after a warm-up)")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if not (a.fetch or a.reads):
        ap.error("--fetch or --reads is required")
    rec = summarise(a.fetch, a.write, a.valu, a.copy_mib, a.batches, a.packets, a.hits, a.reads, a.last_only)
    rec["command"] = a.command
    rec["fields"] = a.fields
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
