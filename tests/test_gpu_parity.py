"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, plus exact device-function checks."""
import numpy as np
import pytest
from scipy import special, stats

import oracle
import workloads as W
from stats_util import chi2_two_sample

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11603_amd import thor
    t = thor.Transport(0)
    yield t
    t.close()


# ------------------------------------------------------------ device functions
def test_voigt_fp64_vs_faddeeva(T):
    _say("voigt fp64")
    a = np.logspace(-6, np.log10(5e-2), 30)
    x = np.concatenate([np.linspace(0, 10, 2001), np.logspace(1, 4, 200)])
    A, X = np.meshgrid(a, np.concatenate([x, -x[1:]]), indexing="ij")
    got = T.voigt(A, X, "fp64")
    ref = special.wofz(X + 1j * A).real
    rel = np.abs(got / ref - 1)
    assert rel.max() < 1e-10, rel.max()
    orc = oracle.voigt(A[::3, ::7], X[::3, ::7])
    assert np.abs(got[::3, ::7] / orc - 1).max() < 1e-12


def test_voigt_fp32_vs_faddeeva(T):
    _say("voigt fp32")
    a = np.logspace(-6, np.log10(5e-2), 30)
    x = np.concatenate([np.linspace(0, 10, 2001), np.logspace(1, 4, 200)])
    A, X = np.meshgrid(a, x, indexing="ij")
    got = T.voigt(A, X, "mixed")
    ref = special.wofz(X.astype(np.float32).astype(float) + 1j * A.astype(np.float32).astype(float)).real
    rel = np.abs(got / ref - 1)
    _say("voigt fp32: max relative error %.3g" % rel.max())
    assert rel.max() < 1e-4            # the FP32 bound of the mixed path
    assert rel.max() < 2e-5            # what the one-form evaluation states


def test_xcw_b25_device(T):
    """x_cw by the Appendix A.2 quartic on the device: FP64 equals the
    oracle's quartic to rounding; the FP32 form with the bit-level logarithm
    stays within 2e-6 of it; both within 0.6 % of the exact Lambert-W x_cw."""
    _say("xcw b25")
    a = np.logspace(np.log10(1.5e-5), -2, 4001)
    b25 = oracle.xcw(a, "b25")
    g64 = T.xcw(a, "fp64")
    g32 = T.xcw(a.astype(np.float32).astype(np.float64), "mixed")
    assert np.abs(g64 / b25 - 1).max() < 1e-13
    b25_32 = oracle.xcw(a.astype(np.float32).astype(np.float64), "b25")
    assert np.abs(g32 / b25_32 - 1).max() < 2e-6, np.abs(g32 / b25_32 - 1).max()
    exact = oracle.xcw(a)
    assert np.abs(g32 / exact - 1).max() < 6e-3


@pytest.mark.parametrize("x,a", [(0.0, 1e-3), (1.0, 1e-3), (2.2, 4.7e-4), (2.3, 4.7e-4), (3.0, 1e-2),
                                 (6.0, 1e-4), (-15.0, 4.7e-4), (40.0, 5e-5)])
def test_upar_fp64_same_seed_as_oracle(T, x, a):
    _say("upar fp64 x=%g a=%g" % (x, a))
    n = 4000
    ug, tg = T.sample_upar(x, a, n, seed=17, event=3, precision="fp64")
    uo, to = oracle.sample_upar(x, a, n, seed=17, event=3)
    same = tg == to
    assert same.mean() > 0.999
    assert np.all(np.abs(ug[same] - uo[same]) <= 1e-9 * (1 + np.abs(uo[same])))


@pytest.mark.parametrize("x,a", [(0.5, 1e-3), (2.0, 4.7e-4), (3.0, 1e-3), (8.0, 1e-4), (25.0, 4.7e-4)])
def test_upar_fp32_distribution(T, x, a):
    _say("upar fp32 x=%g a=%g" % (x, a))
    ug, tg = T.sample_upar(x, a, 50000, seed=23, precision="mixed")
    uo, _ = oracle.sample_upar(x, a, 20000, seed=99)
    assert np.all(np.isfinite(ug))
    assert stats.ks_2samp(ug, uo).pvalue > 1e-3
    assert abs(tg.mean() / oracle.upar_expected_trials(x, a) - 1) < 0.03


# ------------------------------------------------------------ static sphere (tau0 = 1e5)
@pytest.fixture(scope="module")
def sphere_oracle():
    wl = W.sphere()
    return wl, oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, wl["n_packets"], records=True)


def test_sphere_same_seed_trajectories(T, sphere_oracle):
    """500 packets, seed 1, FP64 plain path: per-packet histories follow the
    oracle's; mean scattering count within 1 %."""
    from paper_2507_11603_amd import thor
    wl, ref = sphere_oracle
    _say("sphere same seed plain fp64")
    gpu = thor.run(wl, precision="fp64", path="plain", records=True)
    g, r = gpu["records"], ref["records"]
    assert gpu["stats"]["escaped"] == 500 and gpu["stats"]["capped"] == 0
    frac = np.mean(g["n_res"] == r["n_res"])
    _say("identical histories: %.3f" % frac)
    assert frac > 0.9
    assert abs(g["n_res"].mean() / r["n_res"].mean() - 1) < 0.01
    assert gpu["stats"]["n_res"] == g["n_res"].sum()


@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp64", "persistent"), ("mixed", "persistent")])
def test_sphere_spectrum_chi2(T, sphere_oracle, precision, path):
    """Independent seeds: the GPU escape spectrum (20000 packets) and the
    oracle's (500 packets, seed 1) pass a two-sample chi^2 test at p > 0.01."""
    from paper_2507_11603_amd import thor
    wl, ref = sphere_oracle
    _say("sphere chi2 %s %s" % (precision, path))
    src = dict(wl["src"], seed=1001)
    gpu = thor.run(dict(wl, src=src), n=20000, precision=precision, path=path)
    assert gpu["stats"]["escaped"] == 20000
    chi2, dof, p = chi2_two_sample(gpu["spectrum"], ref["spectrum"])
    _say("chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01


def test_persistent_matches_plain_records(T):
    from paper_2507_11603_amd import thor
    wl = W.sphere(tau0=1e4, n_packets=3000)
    _say("persistent vs plain records")
    a = thor.run(wl, precision="fp64", path="plain", records=True)
    b = thor.run(wl, precision="fp64", path="persistent", records=True)
    assert np.array_equal(a["records"]["n_res"], b["records"]["n_res"])
    assert np.array_equal(a["records"]["dv"], b["records"]["dv"])
    assert np.array_equal(a["spectrum"], b["spectrum"])


def test_bounded_steps_resume_exactly(T):
    """Persistent path in bounded steps of 2 interactions per lane: the
    records equal those of one unbounded launch (counter-keyed RNG)."""
    from paper_2507_11603_amd import thor
    wl = W.sphere(tau0=1e3, n_packets=5000)
    _say("bounded resume")
    ref = thor.run(wl, precision="fp64", path="persistent", records=True)
    t = thor.Transport(0)
    try:
        t.load(wl["geom"])
        t.emit(wl["src"], 5000, 0)
        calls = 0
        while True:
            code, st = t.transport(wl["opts"], precision="fp64", path="persistent", records=True,
                                   step_events=2)
            calls += 1
            if code == thor.OK:
                break
            assert calls < 100000
        rec = t.records()
        spec = t.spectrum()
    finally:
        t.close()
    assert calls > 3
    assert np.array_equal(rec["n_res"], ref["records"]["n_res"])
    assert np.array_equal(rec["dv"], ref["records"]["dv"])
    assert np.array_equal(spec, ref["spectrum"])


# ------------------------------------------------------------ expanding shell on a grid
@pytest.fixture(scope="module")
def shell_case():
    wl = W.shell(n_grid=64, n_packets=20000, cube_nb=64)
    ref = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, 20000, records=True)
    return wl, ref


def test_shell_grid_same_seed(T, shell_case):
    from paper_2507_11603_amd import thor
    wl, ref = shell_case
    _say("shell grid same seed")
    gpu = thor.run(wl, precision="fp64", path="plain", records=True)
    g, r = gpu["records"], ref["records"]
    frac = np.mean((g["n_res"] == r["n_res"]) & (g["n_dust"] == r["n_dust"]) & (g["fate"] == r["fate"]))
    _say("identical histories: %.4f" % frac)
    assert frac > 0.98
    for k in ("escaped", "absorbed", "n_res", "n_dust"):
        assert abs(gpu["stats"][k] - ref["stats"][k]) <= 0.01 * ref["stats"][k] + 5, k
    # cube of the same seed: per-voxel agreement where both have signal
    cg, co = gpu["cube"].astype(float), ref["cube"]
    assert abs(cg.sum() / co.sum() - 1) < 0.01


@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("mixed", "persistent")])
def test_shell_grid_chi2(T, shell_case, precision, path):
    from paper_2507_11603_amd import thor
    wl, ref = shell_case
    _say("shell grid chi2 %s %s" % (precision, path))
    src = dict(wl["src"], seed=1002)
    gpu = thor.run(dict(wl, src=src), n=200000, precision=precision, path=path, records=True)
    chi2, dof, p = chi2_two_sample(gpu["spectrum"], ref["spectrum"])
    _say("spectrum chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01
    fe_g = gpu["stats"]["escaped"] / 200000
    fe_o = ref["stats"]["escaped"] / 20000
    assert abs(fe_g - fe_o) < 4 * np.sqrt(fe_o * (1 - fe_o) / 20000)
    # scattering-count distribution (the mean is dominated by rare packets
    # trapped near line centre, so compare the binned distribution instead)
    edges = np.array([0, 1, 2, 3, 4, 6, 8, 12, 16, 32, 64, 256, 1e9])
    hg = np.histogram(gpu["records"]["n_res"], edges)[0]
    ho = np.histogram(ref["records"]["n_res"], edges)[0]
    chi2, dof, p = chi2_two_sample(hg, ho)
    _say("n_res distribution chi2 %.1f dof %d p %.3f; max n_res gpu %d oracle %d"
         % (chi2, dof, p, gpu["records"]["n_res"].max(), ref["records"]["n_res"].max()))
    assert p > 0.01


def test_shell_seed_pass_matches_inline_peel(T, shell_case):
    """Peel rays through the seed buffer and the peel pass, with a buffer so
    small that transport stops and resumes many times, against rays marched
    inline by the scattering lane: identical packet histories, and the same
    cube up to the order of the float additions (both march each ray's cells
    in the same order with the same arithmetic).  The two kernels are
    separate instantiations, so the compiler may fuse multiply-adds
    differently: final frequencies agree to rounding, not bit for bit."""
    import torch
    from paper_2507_11603_amd import thor
    wl, _ = shell_case
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    _say("shell seed pass vs inline peel (%d CUs)" % n_cu)
    kw = dict(path="persistent", records=True, waves_per_cu=1)
    a = thor.run(wl, precision="fp64", inline_peel=True, **kw)
    b = thor.run(wl, precision="fp64", seed_slots=128 * n_cu, **kw)
    _say("passes %d, peel visits inline %d seeds %d" % (b["stats"]["passes"], a["stats"]["peel_visits"],
                                                         b["stats"]["peel_visits"]))
    assert a["stats"]["passes"] == 1 and b["stats"]["passes"] > 1
    for k in ("n_res", "n_dust", "fate"):
        assert np.array_equal(a["records"][k], b["records"][k]), k
    da, db = a["records"]["dv"], b["records"]["dv"]
    _say("dv: %d of %d differ, max relative difference %.3g"
         % (np.count_nonzero(da != db), da.size, np.max(np.abs(da - db) / np.maximum(np.abs(da), 1.0))))
    assert np.allclose(db, da, rtol=1e-9, atol=1e-3)      # cm/s
    assert a["stats"]["peel_contrib"] == b["stats"]["peel_contrib"]
    ca, cb = a["cube"].astype(np.float64), b["cube"].astype(np.float64)
    assert np.allclose(cb, ca, rtol=1e-5, atol=1e-6 * ca.max())
    # rays whose pixel is outside the cube are dropped before marching on
    # the seed path, so it visits no more cells than the inline march
    assert b["stats"]["peel_visits"] <= a["stats"]["peel_visits"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_wide_turns_same_histories(T, precision):
    """Wide turns (a wave with few live packets evaluates the draws of their
    next events on its idle lanes first) change only which lane evaluates
    the draws: the records equal those of a run without wide turns bit for
    bit, packets trapped near line centre included.  128^3 shell, 1e6
    packets: six of them scatter 3e4-1.3e5 times, alone at the end."""
    from paper_2507_11603_amd import thor
    wl = W.shell(n_packets=1_000_000)
    _say("wide turns on/off, shell 128^3, %s" % precision)
    runs = {w: thor.run(wl, precision=precision, path="persistent", records=True, wide_lanes=w)
            for w in (-1, 16, 1)}
    a = runs[-1]
    _say("n_res max %d; kernel ms off %.1f, 16 lanes %.1f, 1 lane %.1f"
         % (a["records"]["n_res"].max(), a["stats"]["kernel_ms"], runs[16]["stats"]["kernel_ms"],
            runs[1]["stats"]["kernel_ms"]))
    assert a["records"]["n_res"].max() > 10000
    # the longest history (interactions, the absorbing one included), and the
    # tail kernel's share of the interactions
    rec = a["records"]
    ev = rec["n_res"].astype(np.int64) + rec["n_dust"] + (rec["fate"] == 2)
    for w in (-1, 16, 1):
        assert runs[w]["stats"]["max_events"] == ev.max(), w
    assert runs[-1]["stats"]["tail_events"] == 0 and runs[-1]["stats"]["tail_ms"] == 0.0
    assert 0 < runs[16]["stats"]["tail_events"] <= a["stats"]["n_res"] + a["stats"]["n_dust"]
    for w in (16, 1):
        b = runs[w]
        for k in ("n_res", "n_dust", "fate", "dv"):
            assert np.array_equal(a["records"][k], b["records"][k]), (w, k)
        # (main_visits may differ: a segment whose event waits for a new run
        # of seed slots is marched again at the next turn, and wide turns end
        # turns at other points)
        for k in ("n_res", "n_dust", "upar_trials", "peel_contrib", "peel_cut", "peel_visits"):
            assert a["stats"][k] == b["stats"][k], (w, k)
        assert np.array_equal(a["spectrum"], b["spectrum"])        # unit weights: exact sums
        # the same contributions, added by float32 atomics in another order: a
        # voxel summing n positive terms may move by up to n * 6e-8 relative
        # (n reaches 1e4 here)
        ca, cb = a["cube"].astype(np.float64), b["cube"].astype(np.float64)
        big = ca > 1e-3 * ca.max()
        _say("cube: total %.3g relative, max %.3g relative over voxels above 1e-3 of the peak"
             % (abs(cb.sum() / ca.sum() - 1), np.max(np.abs(cb[big] - ca[big]) / ca[big])))
        assert abs(cb.sum() / ca.sum() - 1) < 1e-5
        assert np.allclose(cb, ca, rtol=2e-3, atol=1e-5 * ca.max())


# ------------------------------------------------------------ edge cases and errors
def test_edge_cases(T):
    from paper_2507_11603_amd import thor
    _say("edge cases")
    wl = W.sphere(tau0=1e3, n_packets=1)
    one = thor.run(wl, n=1, records=True)
    assert one["stats"]["emitted"] == 1 and len(one["records"]) == 1
    ragged = thor.run(wl, n=1037, first_id=5, path="persistent", records=True)
    assert ragged["stats"]["escaped"] == 1037
    assert np.all(np.isfinite(ragged["records"]["dv"]))
    t = thor.Transport(0)
    try:
        t.load(wl["geom"])
        code, st = t.transport(wl["opts"])          # nothing emitted: no-op
        assert code == thor.OK and st["emitted"] == 0
        t.emit(wl["src"], 0, 0)                      # empty batch
        with pytest.raises(thor.ThorError) as e:
            t.transport(dict(wl["opts"], spectrum=dict(nb=0, lo=0.0, hi=1.0)))
        assert e.value.code == -1
        with pytest.raises(thor.ThorError):
            t.load(dict(wl["geom"], r_outer=-1.0))
        with pytest.raises(thor.ThorError):
            t.emit(dict(wl["src"], kind="cell_n2"), 10, 0)
    finally:
        t.close()
