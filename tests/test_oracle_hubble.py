"""Oracle pins for the Hubble flow on grids (Section 2.2 frame of the gas,
Section 3.4 sub-cell stepping, the 5 A stop of Section 6.3) in a uniform
static box expanding about its centre, line-centre source at the centre."""
import numpy as np
from scipy import integrate, special

import oracle
import workloads as W


def _tau_to(wl, s):
    """Line optical depth from the source to distance s: the gas-frame
    offset of a photon emitted at line centre is -H s', so tau(s) =
    n sigma0 int_0^s H(a, H s'/v_th) ds' (the profile is even)."""
    g = wl["geom"]
    v, a, sig0 = oracle.line_params(float(g["T_field"].flat[0]))
    n, H = float(g["n_HI_field"].flat[0]), g["hubble"]
    y = H * s / v
    val, _ = integrate.quad(lambda t: special.wofz(t + 1j * a).real, 0.0, y, limit=400, points=[0.0, 1.0, 3.0])
    return n * sig0 * v / H * val


def test_unscattered_photons_stop_by_redshift():
    """A photon that never scatters recedes from the gas at H per unit length:
    it stops by the redshift rule (fate 4, not through a face) after
    stop_dv / H plus at most a cell diagonal (the rule is checked at cell
    faces), with its lab-frame frequency unchanged; the fraction that never
    scatters is exp(-tau(stop_dv / H)) within 4 binomial sigma."""
    n = 3000
    wl = W.hubble_box(n_packets=n)
    r = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, 8, records=True)
    rec = r["records"]
    free = rec["n_res"] == 0
    assert np.all(rec["fate"] == 4)
    assert r["stats"]["redshifted"] == n and r["stats"]["handed_off"] == 0
    assert np.all(rec["dv"][free] == 0.0)
    s_stop = wl["geom"]["stop_dv"] / wl["geom"]["hubble"]
    p = np.exp(-_tau_to(wl, s_stop))
    f = free.mean()
    assert 0.2 < p < 0.8
    assert abs(f - p) < 4 * np.sqrt(p * (1 - p) / n), (f, p)


def test_redshift_stop_distance():
    """Nearly transparent box, no scattering: with the stop at 12.3 Mpc every
    packet stops by redshift before reaching a face 15 Mpc away.  With the
    stop at 16 Mpc a packet stops first only if its face lies beyond the stop
    distance (plus at most a cell diagonal, as the rule is checked at cell
    faces): the fraction stopping lies between the geometric probabilities
    P(15 Mpc / max|k_i| > 16 Mpc + diagonal) and P(... > 16 Mpc) of an
    isotropic direction (sampled here with numpy)."""
    n = 4000
    wl = W.hubble_box(n_HI=1e-16, n_packets=n)
    g = wl["geom"]
    half = (g["hi"][0] - g["lo"][0]) / 2
    diag = np.sqrt(3) * 2 * half / 32
    r = oracle.run_threaded(g, wl["src"], wl["opts"], 0, n, 8, records=True)
    assert np.all(r["records"]["n_res"] == 0) and np.all(r["records"]["fate"] == 4)
    g2 = dict(g, stop_dv=1600.0e5)
    s_stop = g2["stop_dv"] / g2["hubble"]
    r2 = oracle.run_threaded(g2, wl["src"], wl["opts"], 0, n, 8, records=True)
    f = np.mean(r2["records"]["fate"] == 4)
    assert np.all(np.isin(r2["records"]["fate"], (1, 4)))
    k = np.random.default_rng(5).normal(size=(1_000_000, 3))
    m = np.abs(k / np.linalg.norm(k, axis=1)[:, None]).max(axis=1)
    lo, hi = np.mean(half / m > s_stop + diag), np.mean(half / m > s_stop)
    sig = np.sqrt(hi * (1 - hi) / n)
    assert lo - 4 * sig <= f <= hi + 4 * sig, (lo, f, hi)
    assert 0.02 < f < 0.98


def test_emission_peel_through_the_hubble_flow():
    """The +z emission ray of a packet that then escapes unscattered is the
    only contribution in the cube (one pixel, one 0.01 km/s bin at dv = 0):
    1/(4 pi) exp(-tau) with tau = n sigma0 int H(a, H s/v_th) ds from the
    centre to the face, the sub-cell midpoint sums within 2e-3 of the
    quadrature."""
    wl = W.hubble_box(n_packets=1)
    g = wl["geom"]
    half = (g["hi"][2] - g["lo"][2]) / 2
    want = np.exp(-_tau_to(wl, half)) / (4 * np.pi)
    done = 0
    for pid in range(40):
        r = oracle.run(g, wl["src"], wl["opts"], pid, 1, records=True)
        if r["records"]["n_res"][0] != 0:
            continue
        c = r["cube"].ravel()[0]
        assert abs(c / want - 1) < 2e-3, (pid, c, want)
        done += 1
    assert done >= 5
