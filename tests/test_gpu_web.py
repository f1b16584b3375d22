"""Cosmic-web grid (log-normal density, thermal emission proportional to
n_HI^2, fixed core skipping at x_crit = 3, three axis observers): GPU vs
oracle parity, and the precision form's error against FP64."""
import numpy as np
import pytest

import oracle
import workloads as W
from stats_util import chi2_two_sample, chi2_weighted

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def web64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    f = W.web_fields(64)
    wl = W.web(n_grid=64, fields=f, cube_npix=32, cube_nb=50)
    # six chunks of 500 packets give an error bar for the heavy-tailed peel estimator
    parts = [oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 500 * i, 500, records=True, workers=12)
             for i in range(6)]
    ref = {"spectrum": sum(p["spectrum"] for p in parts), "cube": sum(p["cube"] for p in parts),
           "records": np.concatenate([p["records"] for p in parts]),
           "stats": {k: sum(p["stats"][k] for p in parts) for k in parts[0]["stats"]},
           "sb_chunks": np.array([p["cube"].sum(axis=(1, 2, 3)) / 500 for p in parts])}
    return wl, ref


def test_web_same_seed(web64):
    from paper_2507_11603_amd import thor
    wl, ref = web64
    _say("web same seed")
    gpu = thor.run(wl, n=3000, precision="fp64", path="plain", records=True)
    g, r = gpu["records"], ref["records"]
    frac = np.mean(g["n_res"] == r["n_res"])
    _say("identical histories %.3f; mean n_res gpu %.2f oracle %.2f" % (frac, g["n_res"].mean(), r["n_res"].mean()))
    assert frac > 0.8
    assert abs(g["n_res"].mean() / r["n_res"].mean() - 1) < 0.01
    assert gpu["stats"]["handed_off"] == 3000 and gpu["stats"]["escaped"] == 3000
    assert abs(gpu["cube"].sum() / ref["cube"].sum() - 1) < 0.01


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_web_seed_pass_matches_inline_peel(web64, precision):
    """Three observers (+x, +y, +z): peel rays through the seed buffer and the
    peel pass (FP32 rays read the per-axis pencil records) against rays
    marched inline by the scattering lane, on the same packets.  Histories are
    identical; FP64 cubes agree to the order of float additions, FP32 cubes to
    the rounding of the pencil records' derived quantities."""
    import torch
    from paper_2507_11603_amd import thor
    wl, _ = web64
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    _say("web seed pass vs inline peel, %s" % precision)
    kw = dict(n=3000, precision=precision, path="persistent", records=True, waves_per_cu=1)
    a = thor.run(wl, inline_peel=True, **kw)
    b = thor.run(wl, seed_slots=3 * 128 * n_cu, **kw)
    assert b["stats"]["passes"] > 1
    for k in ("n_res", "n_dust", "fate"):
        assert np.array_equal(a["records"][k], b["records"][k]), k
    ca, cb = a["cube"].astype(np.float64), b["cube"].astype(np.float64)
    rel = np.abs(cb - ca).sum() / ca.sum()
    _say("passes %d; cube L1 relative difference %.3g; per observer sums %s vs %s"
         % (b["stats"]["passes"], rel, cb.sum(axis=(1, 2, 3)), ca.sum(axis=(1, 2, 3))))
    tol = 1e-5 if precision == "fp64" else 1e-4
    assert np.allclose(cb, ca, rtol=tol, atol=tol * ca.max())


@pytest.mark.parametrize("precision,path", [("fp64", "persistent"), ("mixed", "persistent")])
def test_web_chi2(web64, precision, path):
    from paper_2507_11603_amd import thor
    wl, ref = web64
    _say("web chi2 %s %s" % (precision, path))
    gpu = thor.run(dict(wl, src=dict(wl["src"], seed=1003)), n=30000, precision=precision, path=path)
    chi2, dof, p = chi2_two_sample(gpu["spectrum"], ref["spectrum"])
    _say("spectrum chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01
    # total peeled flux per observer: oracle chunk error bar (the GPU sample is
    # ten times larger, so its own error adds ~1/sqrt(10) of the oracle's)
    mean = ref["sb_chunks"].mean(axis=0)
    err = ref["sb_chunks"].std(axis=0, ddof=1) / np.sqrt(len(ref["sb_chunks"]))
    tot = gpu["cube"].sum(axis=(1, 2, 3)) / 30000
    _say("peel flux per packet gpu %s oracle %s +- %s" % (tot, mean, err))
    assert np.all(np.abs(tot - mean) < 4 * err * np.sqrt(1.1) + 1e-12), (tot, mean, err)


def test_precision_form_error_report(web64):
    """Mixed precision (FP32 Voigt, direction, redistribution; FP64 position,
    distances, tau) against the FP64 GPU path on the same 200000 packets:
    spectrum chi^2, SB-map error and scattering-count drift (printed and
    bounded)."""
    from paper_2507_11603_amd import thor
    wl, _ = web64
    n = 200000
    a = thor.run(wl, n=n, precision="fp64", path="persistent", records=True)
    b = thor.run(wl, n=n, precision="mixed", path="persistent", records=True)
    chi2, dof, p = chi2_two_sample(a["spectrum"], b["spectrum"])
    da, db = a["records"]["n_res"].astype(float), b["records"]["n_res"].astype(float)
    drift = db.mean() / da.mean() - 1
    same = np.mean(da == db)
    sa = a["cube"].sum(axis=3).astype(float)
    sb = b["cube"].sum(axis=3).astype(float)
    l1 = np.abs(sa - sb).sum() / sa.sum()
    _say("precision report: spectrum chi2 %.1f dof %d p %.3f; n_res drift %.4f; identical histories %.3f; "
         "SB-map L1 rel %.4f; escaped fp64 %d mixed %d" % (chi2, dof, p, drift, same, l1,
                                                         a["stats"]["escaped"], b["stats"]["escaped"]))
    assert p > 0.001
    assert abs(drift) < 0.01
