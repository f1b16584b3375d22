"""Pins of the oracle's Mg II doublet (Section 2.4: a doublet's opacity is the
sum of its transitions, each scattering stays in the line it was absorbed in;
Section 4's doublet test: a sphere with a linear outflow lit by a flat
continuum) against things other than the oracle:

* photons that leave the centre of the outflowing sphere radially without
  scattering do so with probability exp(-tau(dv)), tau from quadrature of the
  two Voigt profiles (scipy's Faddeeva function) over the velocity field;
* with the h line far off resonance the doublet reduces to the k line alone;
* photons at the h line's centre stay symmetric about it;
* the generator's line ratio and flat continuum.
"""
import os

import numpy as np
import pytest
from scipy import special, stats

import oracle
import workloads as W

KMS = 1e5
C_LIGHT = 2.99792458e10
E_CHARGE = 4.80320471e-10
M_ELECTRON = 9.1093837015e-28
K_BOLTZ = 1.380649e-16
M_MG = 24.305 * 1.66053906660e-24
# Mg II k (2P3/2) and h (2P1/2): wavelength (cm), A (1/s), f (Morton 2003)
LINES = [(2796.352e-8, 2.60e8, 0.6155), (2803.531e-8, 2.57e8, 0.3058)]


def _threads():
    return max(1, min(8, os.cpu_count() or 1))


def _sigma(dv_gas, T):
    """Doublet cross-section (cm^2) at gas-frame offset dv_gas (cm/s) from
    the k line, written from the line data: each line's Voigt profile about
    its own centre, in its own Doppler units."""
    vth = np.sqrt(2 * K_BOLTZ * T / M_MG)
    lam_k = LINES[0][0]
    out = 0.0
    for lam, A, f in LINES:
        dnu = vth / lam
        a = A / (4 * np.pi * dnu)
        s0 = f * np.sqrt(np.pi) * E_CHARGE ** 2 / (M_ELECTRON * C_LIGHT * dnu)
        nu_rel = (1 + dv_gas / C_LIGHT) * (lam / lam_k)      # nu / nu_line
        x = (nu_rel - 1) * C_LIGHT / vth
        out = out + s0 * special.wofz(x + 1j * a).real
    return out


def test_species_constants():
    """Mg II k at 1e4 K: v_th = sqrt(2kT/m_Mg) = 2.6157 km/s, and the
    integrated cross-section sigma0 v_th sqrt(pi) = pi e^2 f lambda / (m_e c)."""
    vth, a, s0 = oracle.species_params("mg2", 1e4)
    lam, A, f = LINES[0]
    assert abs(vth / KMS - 2.6157) < 2e-4
    assert abs(s0 * vth * np.sqrt(np.pi) / (np.pi * E_CHARGE ** 2 * f * lam / (M_ELECTRON * C_LIGHT)) - 1) < 1e-12
    assert abs(a * 4 * np.pi * vth / (A * lam) - 1) < 1e-12


@pytest.fixture(scope="module")
def outflow_run():
    n = 16000
    wl = W.mg2_sphere(n_packets=n, v_max_kms=500.0)
    r = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, _threads(), records=True)
    return wl, n, r


def test_unscattered_fraction_matches_quadrature(outflow_run):
    """N_MgII = 10^14.5, T = 1e4 K, v = 500 km/s r/R, flat continuum over
    -1500..1000 km/s from the centre: a packet leaves unscattered with
    probability exp(-tau), tau(dv) = (N / v_max) int_0^v_max sigma(dv - v) dv
    (radial flight through the linear flow).  Per 50 km/s bin, the count of
    unscattered packets (their final dv is the emitted one) against
    N p_b: chi^2 p > 0.001 and every |z| < 4.5.  The deficit covers both
    lines' blue sides, so their strengths, widths and separation are pinned."""
    wl, n, r = outflow_run
    rec = r["records"]
    N = 10 ** 14.5
    vmax = 500.0 * KMS
    lo, hi = -1500.0 * KMS, 1000.0 * KMS
    edges = np.linspace(lo, hi, 51)
    obs, _ = np.histogram(rec["dv"][(rec["n_res"] == 0) & (rec["n_dust"] == 0)], edges)

    # tau(dv) = (N / v_max) [S(dv) - S(dv - v_max)], S the running integral of
    # sigma over a grid 50 points per thermal width; p_b the mean of
    # exp(-tau) over the bin (the edges of the resonant band are a few
    # thermal widths wide)
    du = 0.05 * KMS
    u = np.arange(lo - vmax - du, hi + du, du)
    S = np.concatenate([[0.0], np.cumsum(0.5 * (_sigma(u[1:], 1e4) + _sigma(u[:-1], 1e4)) * du)])
    fine = np.arange(lo + 0.125 * KMS, hi, 0.25 * KMS)
    tau = N / vmax * (np.interp(fine, u, S) - np.interp(fine - vmax, u, S))
    pe = np.exp(-tau)
    p = np.array([pe[(fine >= a) & (fine < b)].mean() for a, b in zip(edges[:-1], edges[1:])]) / 50.0
    z = (obs - n * p) / np.sqrt(n * p * (1 - p))
    chi2 = float(np.sum(z ** 2))
    pval = stats.chi2.sf(chi2, len(p))
    print("unscattered: chi2 %.1f / %d, p %.3g, max |z| %.2f; min p_esc %.3f" % (chi2, len(p), pval,
                                                                                   np.abs(z).max(), p.min() * 50))
    assert pval > 1e-3 and np.abs(z).max() < 4.5
    # the P Cygni shape of the k line: deficit blueward, excess redward
    spec = r["spectrum"].reshape(50, -1).sum(axis=1)
    centres = 0.5 * (edges[:-1] + edges[1:])
    level = n / 50.0
    blue = (centres > 50 * KMS) & (centres < 450 * KMS)
    red = (centres < -50 * KMS) & (centres > -450 * KMS)
    assert spec[blue].mean() < 0.8 * level < level < spec[red].mean()
    assert r["stats"]["escaped"] == n


def test_doublet_reduces_to_k_line_alone():
    """A static sphere (tau0 of the k line near 1e3) lit at the k line's
    centre: the h line, 768 km/s away, adds an opacity ~1e-8 of the k line's,
    so the doublet follows the k line alone packet by packet (same seed)."""
    n = 1500
    kw = dict(log_N=15.0, v_max_kms=0.0, spectrum="delta", dv0_kms=0.0, n_packets=n, continuum_kms=(-60, 60),
              nb=60)
    ra = oracle.run_threaded(**_args(W.mg2_sphere(line="mg2", **kw), n), records=True)
    rb = oracle.run_threaded(**_args(W.mg2_sphere(line="mg2k", **kw), n), records=True)
    a, b = ra["records"], rb["records"]
    same = (a["n_res"] == b["n_res"]) & (a["dv"] == b["dv"])
    assert same.mean() > 0.99, same.mean()
    assert a["n_res"].mean() > 100


def _args(wl, n):
    return dict(geom=wl["geom"], src=wl["src"], opts=wl["opts"], first_id=0, n=n, threads=_threads())


def test_h_line_photons_stay_about_the_h_line():
    """Lit at the h line's centre (c (lambda_k/lambda_h - 1) = -767.6 km/s
    from k), packets scatter in h and escape symmetrically about its centre:
    the mirrored offsets pass a two-sample test and the mean is within 4
    standard errors of it."""
    n = 3000
    c_h = C_LIGHT * (LINES[0][0] / LINES[1][0] - 1.0)
    wl = W.mg2_sphere(log_N=15.0, v_max_kms=0.0, spectrum="delta", dv0_kms=c_h / KMS, n_packets=n,
                      continuum_kms=(-860, -680), nb=90)
    r = oracle.run_threaded(**_args(wl, n), records=True)
    rec = r["records"]
    d = rec["dv"] - c_h
    assert rec["n_res"].mean() > 30
    assert abs(d.mean()) < 4 * d.std() / np.sqrt(n)
    assert stats.ks_2samp(d, -d).pvalue > 1e-3
    assert np.abs(d).max() < 40 * KMS


def test_doublet_emission_ratio_and_flat_continuum():
    """The generator: a doublet source emits in h with probability
    f_h / (f_k + f_h) (binomial, 4 sigma), at the h line's centre; a flat
    continuum is uniform over dv0 +- sigma_v (KS)."""
    n = 20000
    wl = W.mg2_sphere(spectrum="delta", dv0_kms=0.0, n_packets=n)
    src = dict(wl["src"], lines=1)
    e = oracle.emit(wl["geom"], src, 0, n)
    c_h = C_LIGHT * (LINES[0][0] / LINES[1][0] - 1.0)
    at_h = np.isclose(e["dv"], c_h, rtol=0, atol=1.0)
    assert np.all(at_h | (e["dv"] == 0.0))
    p = LINES[1][2] / (LINES[0][2] + LINES[1][2])
    assert abs(at_h.mean() - p) < 4 * np.sqrt(p * (1 - p) / n)
    wf = W.mg2_sphere(n_packets=n)
    ef = oracle.emit(wf["geom"], wf["src"], 0, n)
    lo, hi = -1500 * KMS, 1000 * KMS
    assert stats.kstest((ef["dv"] - lo) / (hi - lo), "uniform").pvalue > 1e-3
