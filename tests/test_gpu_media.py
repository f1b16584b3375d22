"""GPU parity for the Section 4 validation media: dust escape from a slab
against the closed form at the paper's configuration and against the
oracle, and the linear-outflow sphere against the oracle."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from stats_util import chi2_two_sample
from test_oracle_media import fesc_slab

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


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_slab_dust_escape_matches_closed_form(gpu, precision):
    """T = 20 K, tau0 = 1e6 (a tau0 = 1.05e4), albedo 0, line-centre source
    (the paper's dust test): escape fractions at b = (a tau0)^(1/3) tau_d =
    0.25 ... 2 (FP64: 0.5 and 1) within 0.02 (+ 3 sigma) of the closed form;
    5000 packets per b."""
    _, a, _ = oracle.line_params(20.0)
    n = 5000
    for b in ((0.25, 0.5, 1.0, 2.0) if precision == "mixed" else (0.5, 1.0)):
        tau_d = b / (a * 1e6) ** (1 / 3)
        r = gpu.run(W.dusty_slab(tau0=1e6, tau_d=tau_d, n_packets=n), precision=precision, path="persistent")
        st = r["stats"]
        f = st["escaped"] / n
        sig = np.sqrt(f * (1 - f) / n)
        an = fesc_slab(a, 1e6, tau_d)
        _say("slab %s b %.2f: f_esc %.4f +- %.4f, closed form %.4f" % (precision, b, f, sig, an))
        assert st["escaped"] + st["absorbed"] == n and st["capped"] == 0
        assert abs(f - an) < 0.02 + 3 * sig


def test_slab_dust_escape_matches_oracle(gpu):
    """tau0 = 1e5 at T = 20 K, b = 1: the GPU's escape fraction (2e4 packets,
    another seed) and the oracle's (800 packets) agree within 4 sigma of
    their difference."""
    _, a, _ = oracle.line_params(20.0)
    tau_d = 1.0 / (a * 1e5) ** (1 / 3)
    wl = W.dusty_slab(tau0=1e5, tau_d=tau_d, n_packets=800)
    ro = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, 800, _threads())
    g = gpu.run(dict(wl, src=dict(wl["src"], seed=1001)), n=20000, precision="mixed", path="persistent")
    fo, fg = ro["stats"]["escaped"] / 800, g["stats"]["escaped"] / 20000
    err = np.sqrt(fo * (1 - fo) / 800 + fg * (1 - fg) / 20000)
    _say("slab b=1 tau0=1e5: gpu %.4f oracle %.4f +- %.4f" % (fg, fo, err))
    assert abs(fg - fo) < 4 * err


def test_outflow_sphere_against_oracle(gpu):
    """Linear outflow v = 200 km/s r/R, N_HI = 2e17, T = 2e4 K: FP64 plain
    path with the oracle's seed follows its histories; mixed persistent
    spectra of another seed pass chi^2 against the oracle's; outflow and
    infall mirror each other on the GPU too."""
    n = 3000
    wl = W.outflow_sphere(N_HI=2e17, v_max_kms=200.0, n_packets=n)
    ro = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, _threads(), records=True)
    g = gpu.run(wl, precision="fp64", path="plain", records=True)
    same = np.mean(g["records"]["n_res"] == ro["records"]["n_res"])
    _say("outflow same seed: identical histories %.3f" % same)
    assert same > 0.9
    assert abs(g["records"]["n_res"].mean() / ro["records"]["n_res"].mean() - 1) < 0.01
    m = gpu.run(dict(wl, src=dict(wl["src"], seed=1001)), n=100000, precision="mixed", path="persistent")
    chi2, dof, p = chi2_two_sample(m["spectrum"], ro["spectrum"])
    _say("outflow mixed 1e5 vs oracle: chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01
    inf = W.outflow_sphere(N_HI=2e17, v_max_kms=-200.0, n_packets=n)
    mi = gpu.run(dict(inf, src=dict(inf["src"], seed=1002)), n=100000, precision="mixed", path="persistent")
    chi2, dof, p = chi2_two_sample(m["spectrum"], mi["spectrum"][::-1])
    _say("outflow vs reversed infall: chi2 %.1f dof %d p %.3f" % (chi2, dof, p))
    assert p > 0.01
