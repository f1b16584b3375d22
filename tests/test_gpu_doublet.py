"""GPU parity of the Mg II doublet (Section 2.4; Section 4's doublet test: a
sphere with a linear outflow lit by a flat continuum) against the oracle,
through the C ABI:

* FP64, the oracle's seed: the histories follow the oracle's;
* mixed precision, another seed: escape spectra pass a two-sample chi^2;
* the unscattered fraction per emitted frequency equals exp(-tau) from
  quadrature of the two Voigt profiles (the same pin as the oracle's);
* with h off resonance the doublet follows the k line alone;
* a doublet source emits in h in the ratio of the oscillator strengths;
* grids refuse the Mg II lines.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from stats_util import chi2_two_sample
from test_oracle_doublet import C_LIGHT, KMS, LINES, _sigma

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2507_11603_amd import thor
    thor.lib()
    return thor


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def outflow_oracle():
    n = 4000
    wl = W.mg2_sphere(n_packets=n, v_max_kms=500.0)
    return wl, n, oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, _threads(), records=True)


@pytest.mark.parametrize("path", ["plain", "persistent"])
def test_doublet_fp64_same_seed(gpu, outflow_oracle, path):
    """FP64 with the oracle's seed and ids: more than 98 % of the histories
    (scattering count and final frequency) are the oracle's."""
    wl, n, ro = outflow_oracle
    rg = gpu.run(wl, n=n, precision="fp64", path=path, records=True)
    a, b = ro["records"], rg["records"]
    same = (a["n_res"] == b["n_res"]) & (np.abs(a["dv"] - b["dv"]) <= 1e-6 * KMS)
    _say("doublet fp64 %s: %.4f identical histories, mean scatterings %.3f vs %.3f"
         % (path, same.mean(), b["n_res"].mean(), a["n_res"].mean()))
    assert same.mean() > 0.98
    assert rg["stats"]["escaped"] == n and rg["stats"]["handed_off"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_doublet_chi2_vs_oracle(gpu, outflow_oracle, precision):
    """Another seed, 1e5 packets on the persistent path: the escape spectrum
    (250 bins, merged) against the oracle's 4000 packets, p > 0.01."""
    wl, n, ro = outflow_oracle
    src = dict(wl["src"], seed=1001)
    rg = gpu.run(dict(wl, src=src), n=100000, precision=precision, path="persistent")
    chi2, dof, p = chi2_two_sample(ro["spectrum"], rg["spectrum"])
    _say("doublet %s chi2 %.1f / %d, p %.3g" % (precision, chi2, dof, p))
    assert p > 0.01


def test_doublet_unscattered_fraction_matches_quadrature(gpu):
    """2e5 packets, mixed precision, persistent path: per 50 km/s bin of the
    emitted frequency, the unscattered count against N exp(-tau) p_bin
    (tau from quadrature of both lines over the linear flow)."""
    n = 200000
    wl = W.mg2_sphere(n_packets=n, v_max_kms=500.0, seed=77)
    rec = gpu.run(wl, n=n, precision="mixed", path="persistent", records=True)["records"]
    N, vmax = 10 ** 14.5, 500.0 * KMS
    lo, hi = -1500.0 * KMS, 1000.0 * KMS
    edges = np.linspace(lo, hi, 51)
    obs, _ = np.histogram(rec["dv"][(rec["n_res"] == 0) & (rec["n_dust"] == 0)], edges)
    du = 0.05 * KMS
    u = np.arange(lo - vmax - du, hi + du, du)
    S = np.concatenate([[0.0], np.cumsum(0.5 * (_sigma(u[1:], 1e4) + _sigma(u[:-1], 1e4)) * du)])
    fine = np.arange(lo + 0.125 * KMS, hi, 0.25 * KMS)
    pe = np.exp(-N / vmax * (np.interp(fine, u, S) - np.interp(fine - vmax, u, S)))
    p = np.array([pe[(fine >= a) & (fine < b)].mean() for a, b in zip(edges[:-1], edges[1:])]) / 50.0
    z = (obs - n * p) / np.sqrt(n * p * (1 - p))
    from scipy import stats
    chi2 = float(np.sum(z ** 2))
    pval = stats.chi2.sf(chi2, len(p))
    _say("doublet unscattered: chi2 %.1f / %d, p %.3g, max |z| %.2f" % (chi2, len(p), pval, np.abs(z).max()))
    assert pval > 1e-3 and np.abs(z).max() < 4.5


def test_doublet_reduces_to_k_line_alone(gpu):
    """Static sphere lit at the k line's centre: the doublet and the k line
    alone give the same histories (FP64, same seed)."""
    n = 3000
    kw = dict(log_N=15.0, v_max_kms=0.0, spectrum="delta", dv0_kms=0.0, n_packets=n, continuum_kms=(-60, 60),
              nb=60)
    ra = gpu.run(W.mg2_sphere(line="mg2", **kw), precision="fp64", path="persistent", records=True)
    rb = gpu.run(W.mg2_sphere(line="mg2k", **kw), precision="fp64", path="persistent", records=True)
    a, b = ra["records"], rb["records"]
    same = (a["n_res"] == b["n_res"]) & (a["dv"] == b["dv"])
    _say("doublet vs k line: %.4f identical" % same.mean())
    assert same.mean() > 0.99 and a["n_res"].mean() > 100


def test_doublet_emission_ratio(gpu):
    """A thin medium (N = 1e8 cm^-2) and a doublet source at line centre: the
    escaping packets sit at the k and h centres in the ratio f_k : f_h."""
    n = 100000
    c_h = C_LIGHT * (LINES[0][0] / LINES[1][0] - 1.0)
    wl = W.mg2_sphere(log_N=8.0, v_max_kms=0.0, spectrum="delta", dv0_kms=0.0, n_packets=n,
                      continuum_kms=(-1000, 100), nb=1100)
    wl["src"]["lines"] = 1
    rec = gpu.run(wl, precision="mixed", path="persistent", records=True)["records"]
    # the few packets that scatter (tau ~ 1e-4) leave the line centres
    rec = rec[rec["n_res"] == 0]
    assert len(rec) > 0.999 * n
    at_h = np.abs(rec["dv"] - c_h) < 1.0 * KMS
    at_k = np.abs(rec["dv"]) < 1.0 * KMS
    assert np.all(at_h | at_k)
    p = LINES[1][2] / (LINES[0][2] + LINES[1][2])
    _say("doublet emission: %.4f in h (expected %.4f)" % (at_h.mean(), p))
    assert abs(at_h.mean() - p) < 4 * np.sqrt(p * (1 - p) / len(rec))


def test_mg2_lines_refused_on_grids(gpu):
    wl = W.shell(n_grid=16, n_packets=10)
    T = gpu.Transport(0)
    try:
        with pytest.raises(gpu.ThorError) as e:
            T.load(dict(wl["geom"], line="mg2"))
        assert "meshless" in str(e.value)
    finally:
        T.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_frequency_presort_changes_only_the_order(gpu, precision):
    """Queue sorted by emitted frequency (presort 2, Section 7.1's
    pre-sorting) on the flat continuum through the Mg II outflow: records,
    spectrum and the physical counters equal those of the queue order."""
    n = 20000
    wl = W.mg2_sphere(n_packets=n, v_max_kms=500.0, seed=5)
    res = []
    for presort in (-1, 2):
        r = gpu.run(wl, n=n, precision=precision, path="persistent", records=True, presort=presort)
        res.append(r)
    a, b = res
    _say("frequency presort %s: %.2f ms of %.2f ms" % (precision, b["stats"]["presort_ms"], b["stats"]["kernel_ms"]))
    assert a["stats"]["presort_ms"] == 0.0 and b["stats"]["presort_ms"] > 0.0
    assert np.array_equal(a["spectrum"], b["spectrum"])
    for k in ("n_res", "n_dust", "fate", "dv"):
        assert np.array_equal(a["records"][k], b["records"][k]), k
    for k in ("emitted", "escaped", "n_res", "main_visits", "upar_trials"):
        assert a["stats"][k] == b["stats"][k], k
