"""Precision form on the 512^3 cosmic-web box (not collected by pytest; run by hand).

    python tests/precision_web512.py oracle OUT.npz [--n 100000]
        the CPU oracle (FP64) on photon ids 0..n-1 (host cores)
    python tests/precision_web512.py gpu ORACLE.npz [--n-big 10000000]
        on the GPU: FP64 and mixed precision on the same n-big packets (the
        precision form's error against FP64), and both on the oracle's ids
        against the oracle

Fields: the numpy recipe of `workloads.web_fields` at 512^3 (seeded), thermal
n_HI^2 emission, x_crit = 3, three axis observers.  The image is binned 64^2
(instead of 512^2) so that the oracle's per-process cubes stay small; the
spectral bins are the workload's 200 over +-1500 km/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import workloads as W  # noqa: E402


def workload():
    return W.web(n_grid=512, fields=W.web_fields(512), cube_npix=64, cube_nb=200)


def sb_maps(cube):
    """Surface-brightness maps: the cube summed over frequency, per observer."""
    return cube.astype(np.float64).sum(axis=3)


def compare(a, b, label):
    """Errors of result b against reference a (same packets or same recipe)."""
    from stats_util import chi2_two_sample
    chi2, dof, p = chi2_two_sample(a["spectrum"], b["spectrum"])
    sa, sb = sb_maps(a["cube"]), sb_maps(b["cube"])
    nz = a["spectrum"] > 0
    return {"label": label, "spectrum_chi2": chi2, "dof": dof, "p": p,
            "spectrum_max_rel_bin_err": float(np.max(np.abs(b["spectrum"][nz] - a["spectrum"][nz]) / a["spectrum"][nz])),
            "sb_l1_rel": float(np.abs(sa - sb).sum() / sa.sum()),
            "sb_total_rel": (sb.sum(axis=(1, 2)) / sa.sum(axis=(1, 2)) - 1).tolist(),
            "scatterings_drift": (b["stats"]["n_res"] + b["stats"]["n_dust"]) / (a["stats"]["n_res"] + a["stats"]["n_dust"]) - 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["oracle", "gpu"])
    ap.add_argument("path")
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--n-big", type=int, default=10_000_000)
    ap.add_argument("--workers", type=int, default=0)
    a = ap.parse_args()
    wl = workload()
    if a.mode == "oracle":
        import oracle
        t0 = time.time()
        r = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, a.n, workers=a.workers or None, records=True)
        np.savez(a.path, spectrum=r["spectrum"], cube=r["cube"], n_res=r["records"]["n_res"],
                 stats=json.dumps({k: int(v) for k, v in r["stats"].items()}), n=a.n)
        print("oracle: %d packets in %.0f s" % (a.n, time.time() - t0), flush=True)
        return
    import torch

    from paper_2507_11603_amd import thor
    ref = np.load(a.path)
    oref = {"spectrum": ref["spectrum"], "cube": ref["cube"], "stats": json.loads(str(ref["stats"]))}
    n = int(ref["n"])
    T = thor.Transport(0)
    T.load(wl["geom"])
    shape = (3, 64, 64, 200)
    out = {}

    def run(nn, first, precision):
        T.reset()
        torch.cuda.synchronize()
        T.emit(wl["src"], nn, first)
        code, st = T.transport(wl["opts"], precision=precision, path="persistent", records=True)
        rec = T.records()
        return {"spectrum": T.spectrum(), "cube": T.cube(shape), "stats": st, "n_res": rec["n_res"].copy()}

    g64 = run(n, 0, "fp64")
    gmx = run(n, 0, "mixed")
    out["fp64_vs_oracle"] = compare(oref, g64, "GPU FP64 vs oracle, %d packets" % n)
    out["mixed_vs_oracle"] = compare(oref, gmx, "GPU mixed vs oracle, %d packets" % n)
    out["fp64_same_histories_as_oracle"] = float(np.mean(g64["n_res"] == ref["n_res"]))
    b64 = run(a.n_big, 0, "fp64")
    bmx = run(a.n_big, 0, "mixed")
    out["mixed_vs_fp64"] = compare(b64, bmx, "GPU mixed vs GPU FP64, same %d packets" % a.n_big)
    out["mixed_same_histories_as_fp64"] = float(np.mean(b64["n_res"] == bmx["n_res"]))
    T.close()
    print(json.dumps(out, indent=1), flush=True)


if __name__ == "__main__":
    main()
