"""Transport-level pins of the oracle against exact results and the analytic
high-optical-depth solutions (Sections 3.4 and 4 of the paper)."""
import os

import numpy as np
import pytest
from scipy import integrate, optimize, special, stats

import oracle
import workloads as W

KPC, KMS = W.KPC, W.KMS


def test_flux_conservation_dust_free():
    """With dust off every packet escapes with its full weight (P7)."""
    wl = W.sphere(tau0=1e4, n_packets=60)
    r = oracle.run(wl["geom"], wl["src"], wl["opts"], 0, 60, records=True)
    st = r["stats"]
    assert st["escaped"] == 60 and st["absorbed"] == 0 and st["capped"] == 0
    assert st["w_escaped"] == 60.0
    assert r["spectrum"].sum() == 60.0           # +-40 v_th holds every photon here
    assert np.all(r["records"]["fate"] == 1)
    assert st["n_res"] == r["records"]["n_res"].sum()


def test_static_sphere_spectrum_symmetric():
    wl = W.sphere(tau0=1e4, n_packets=400)
    r = oracle.run_parallel(wl["geom"], wl["src"], wl["opts"], 0, 400, records=True)
    x = r["records"]["dv"]
    assert abs(np.mean(np.sign(x))) < 5 / np.sqrt(400)


def test_pure_absorber_escape_fraction():
    """Central source in a dusty shell, albedo 0, resonant opacity negligible:
    f_esc = exp(-tau_d) exactly (P8)."""
    tau_d, n = 1.3, 20000
    geom = dict(kind="shell", r_inner=0.5 * KPC, r_outer=KPC, n_HI=1e-12, T=1e4,
                tau_d=tau_d, albedo=0.0)
    src = dict(kind="point", spectrum="delta", dv0=0.0, seed=21)
    opts = dict(phase="dipole", spectrum=dict(nb=10, lo=-1e7, hi=1e7))
    r = oracle.run(geom, src, opts, 0, n)
    p = np.exp(-tau_d)
    k = r["stats"]["escaped"]
    assert r["stats"]["escaped"] + r["stats"]["absorbed"] == n
    assert abs(k - n * p) < 4 * np.sqrt(n * p * (1 - p))


def test_optically_thin_limit():
    """tau0 -> 0: no scatterings and the escaped spectrum is the intrinsic
    Gaussian (P9)."""
    wl = W.sphere(tau0=1e-9, n_packets=5000)
    src = dict(kind="point", spectrum="gauss", dv0=0.0, sigma_v=20 * KMS, seed=9)
    r = oracle.run(wl["geom"], src, wl["opts"], 0, 5000, records=True)
    assert r["stats"]["n_res"] == 0
    z = r["records"]["dv"] / (20 * KMS)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_single_scattering_probability():
    """Static sphere, source at line centre: P(at least one scattering) =
    1 - exp(-tau0 H(a,0)) since the radial optical depth at x = 0 is
    tau0 H(a, 0) (eq. fluxdec with sigma = sigma0 H)."""
    tau0, n = 0.05, 40000
    wl = W.sphere(tau0=tau0, n_packets=n)
    r = oracle.run(wl["geom"], wl["src"], wl["opts"], 0, n, records=True)
    _, a, _ = oracle.line_params(1e4)
    p = 1 - np.exp(-tau0 * np.exp(a * a) * special.erfc(a))
    k = np.count_nonzero(r["records"]["n_res"] > 0)
    assert abs(k - n * p) < 4 * np.sqrt(n * p * (1 - p))


def test_grid_peel_optical_depth_exact():
    """Homogeneous grid, absorbing dust, photons far in the wing: every
    emission peel towards +z sees tau = (k_d + n sigma0 H(a, x)) (z_hi - z0)
    exactly, so the +z cube holds N exp(-tau)/(4 pi) in one voxel (P10)."""
    ng, n = 8, 300
    L = KPC
    dens = np.full((ng, ng, ng), 1e-4, np.float32)
    temp = np.full((ng, ng, ng), 1e4, np.float32)
    zero = np.zeros((ng, ng, ng), np.float32)
    sigma_d = 2.0 / (1e-4 * L)           # tau_d = 1 over half the box
    geom = dict(kind="grid", lo=(-L, -L, -L), hi=(L, L, L), n_HI_field=dens, T_field=temp,
                vx=zero, vy=zero, vz=zero, sigma_d=sigma_d, albedo=0.0)
    dv0 = 3000 * KMS
    src = dict(kind="point", pos=(0.1 * L, -0.3 * L, 0.2 * L), spectrum="delta", dv0=dv0, seed=4)
    opts = dict(phase="dipole", observers=["+z"],
                cube=dict(nx=ng, ny=ng, nb=4, img_lo=(-L, -L), img_hi=(L, L),
                          v_lo=2000 * KMS, v_hi=4000 * KMS),
                spectrum=dict(nb=4, lo=2000 * KMS, hi=4000 * KMS))
    r = oracle.run(geom, src, opts, 0, n)
    vth, a, s0 = oracle.line_params(1e4)
    n_hi = float(np.float32(1e-4))
    H = special.wofz(dv0 / vth + 1j * a).real
    tau = (sigma_d * n_hi + n_hi * s0 * H) * (L - 0.2 * L)
    cube = r["cube"][0]
    nz = np.argwhere(cube > 0)
    ix, iy = int(np.floor((0.1 * L + L) / (2 * L / ng))), int(np.floor((-0.3 * L + L) / (2 * L / ng)))
    assert [tuple(v) for v in nz] == [(iy, ix, 2)]
    # dust absorbs everything scattered, so only emission peels contribute
    assert r["stats"]["n_res"] + r["stats"]["n_dust"] == 0
    want = n * np.exp(-tau) / (4 * np.pi)
    assert abs(cube[iy, ix, 2] / want - 1) < 1e-12


def test_grid_escape_fraction_matches_direction_average():
    """Homogeneous absorbing cube, isotropic point source: the escape fraction is
    the direction average of exp(-k_d l(k)) with l the distance to the cube
    surface, computed here by independent quadrature over the sphere."""
    ng, n = 4, 20000
    L = KPC
    dens = np.full((ng, ng, ng), 1.0, np.float32)
    temp = np.full((ng, ng, ng), 1e4, np.float32)
    zero = np.zeros((ng, ng, ng), np.float32)
    kd = 1.0 / L
    geom = dict(kind="grid", lo=(-L, -L, -L), hi=(L, L, L), n_HI_field=dens, T_field=temp,
                vx=zero, vy=zero, vz=zero, sigma_d=kd, albedo=0.0)
    p0 = np.array([0.3, -0.55, 0.1]) * L
    src = dict(kind="point", pos=tuple(p0), spectrum="delta", dv0=5e4 * KMS, seed=6)
    opts = dict(phase="dipole", spectrum=dict(nb=4, lo=0.0, hi=1e10))
    r = oracle.run(geom, src, opts, 0, n)

    def dist(mu, phi):
        s = np.sqrt(1 - mu * mu)
        k = np.array([s * np.cos(phi), s * np.sin(phi), mu])
        t = np.inf
        for ax in range(3):
            if k[ax] > 0:
                t = min(t, (L - p0[ax]) / k[ax])
            elif k[ax] < 0:
                t = min(t, (-L - p0[ax]) / k[ax])
        return t

    f = integrate.dblquad(lambda phi, mu: np.exp(-kd * dist(mu, phi)), -1, 1, 0, 2 * np.pi,
                          epsabs=1e-10)[0] / (4 * np.pi)
    k = r["stats"]["escaped"]
    assert abs(k - n * f) < 4 * np.sqrt(n * f * (1 - f))


def test_peel_normalisation_spherical():
    """Spherically symmetric medium: the peeled-off flux per steradian towards
    any observer is N / (4 pi) on average (P7).  Error bar from 8 independent
    chunks (the next-event estimator is heavy-tailed)."""
    n = 2000
    wl = W.sphere(tau0=1e3, n_packets=n)
    opts = dict(wl["opts"], observers=["+z", "-x", "+y"],
                cube=dict(nx=1, ny=1, nb=1, img_lo=(-1.0, -1.0), img_hi=(1.0, 1.0),
                          v_lo=-1e9, v_hi=1e9))
    tots = []
    for c in range(8):
        r = oracle.run_parallel(wl["geom"], dict(wl["src"], seed=100 + c), opts, 0, n)
        assert r["stats"]["peel_dropped"] == 0
        tots.append(r["cube"].sum(axis=(1, 2, 3)) * 4 * np.pi / n)
    tots = np.array(tots)
    err = tots.std(axis=0, ddof=1) / np.sqrt(len(tots))
    assert np.all(np.abs(tots.mean(axis=0) - 1) < 5 * err + 0.005), (tots.mean(axis=0), err)


def test_albedo_one_dust_conserves_flux():
    n = 2000
    geom = dict(kind="shell", r_inner=0.0, r_outer=KPC, tau0=1e3, T=1e4, tau_d=2.0,
                albedo=1.0, g_hg=0.73)
    src = dict(kind="point", spectrum="gauss", sigma_v=20 * KMS, seed=8)
    opts = dict(phase="dipole", spectrum=dict(nb=100, lo=-1e8, hi=1e8))
    r = oracle.run(geom, src, opts, 0, n)
    assert r["stats"]["escaped"] == n and r["stats"]["n_dust"] > 0


# Asymptotic (a tau0 >> 1) emergent spectra of a central line-centre source,
# J(x) ~ x^2 g(beta |x|^3 / (a tau0)): the Neufeld slab, g = 1/cosh, beta =
# sqrt(pi^3/54), and the Dijkstra et al. sphere, g = 1/(1 + cosh), beta =
# sqrt(2 pi^3/27) (the Section 4 validation of the paper; the formulas are the
# cited solutions).  y = |x|^3 then has the scale-family density g(y/theta) /
# (Z theta) with theta = a tau0 / beta, Z = pi/2 (slab) or 1 (sphere).
PROFILES = {"slab": (np.sqrt(np.pi ** 3 / 54), lambda u: 1 / np.cosh(u), np.pi / 2),
            "sphere": (np.sqrt(2 * np.pi ** 3 / 27), lambda u: 1 / (1 + np.cosh(u)), 1.0)}


def peak_coefficient(kind):
    """c in x_peak = c (a tau0)^(1/3): the maximum of x^2 g(beta x^3)."""
    beta, g, _ = PROFILES[kind]
    res = optimize.minimize_scalar(lambda x: -x * x * g(beta * x ** 3), bounds=(0.1, 3.0),
                                   method="bounded", options={"xatol": 1e-12})
    return res.x


def fitted_peak(kind, x, n_boot=200, seed=0):
    """Maximum-likelihood fit of the asymptotic profile's one free scale to the
    escaped |x|; returns the peak of the fitted profile and its bootstrap error."""
    beta, g, Z = PROFILES[kind]
    y = np.abs(x) ** 3

    def fit(yy):
        nll = lambda lt: len(yy) * lt - np.sum(np.log(g(yy / np.exp(lt))))
        lt0 = np.log(np.mean(yy))
        return np.exp(optimize.minimize_scalar(nll, bounds=(lt0 - 4, lt0 + 4), method="bounded").x)

    c = peak_coefficient(kind)
    peak = lambda th: c * (beta * th) ** (1 / 3)
    rng = np.random.default_rng(seed)
    boot = [peak(fit(rng.choice(y, len(y)))) for _ in range(n_boot)]
    return peak(fit(y)), np.std(boot)


def _peak_offset(kind, tau0, T, n):
    """(fitted peak / predicted peak - 1, its 1-sigma error) for n packets."""
    wl = W.sphere(tau0=tau0, T=T, n_packets=n, kind=kind)
    r = oracle.run_threaded(wl["geom"], wl["src"], wl["opts"], 0, n, os.cpu_count() or 1, records=True)
    vth, a, _ = oracle.line_params(T)
    x = r["records"]["dv"] / vth
    pk, err = fitted_peak(kind, x)
    pred = peak_coefficient(kind) * (a * tau0) ** (1 / 3)
    return pk / pred - 1, err / pred


def test_peak_coefficients():
    """The maxima of the two asymptotic profiles: 1.0664 (slab) and 0.9310
    (sphere) times (a tau0)^(1/3); the quoted 1.066 and 0.92 round these."""
    assert abs(peak_coefficient("slab") - 1.0664) < 2e-4
    assert abs(peak_coefficient("sphere") - 0.9310) < 2e-4


# a tau0 = 4.7e3: the diffusion solutions depend on a and tau0 only through
# a tau0, which T = 10 K (a = 1.49e-2) reaches at tau0 = 3.16e5, with 30 times
# fewer scatterings per packet than T = 1e4 K at tau0 = 1e7
T_COLD, TAU_COLD = 10.0, 3.16e5


@pytest.mark.slow
def test_slab_asymptotic_peak():
    """Neufeld slab at a tau0 = 4.7e3: the fitted peak within 5 % (+ 2 sigma)
    of 1.066 (a tau0)^(1/3)."""
    d, e = _peak_offset("slab", TAU_COLD, T_COLD, 300)
    assert abs(d) < 0.05 + 2 * e, (d, e)


@pytest.mark.slow
def test_sphere_peaks_converge_with_optical_depth():
    """Dijkstra sphere: at a tau0 = 47 (tau0 = 1e5, T = 1e4 K) the asymptotic
    form does not hold yet and the peak sits well outside it; at a tau0 = 4.7e3
    the fitted peak is within 5 % (+ 2 sigma) of 0.931 (a tau0)^(1/3)."""
    d5, e5 = _peak_offset("sphere", 1e5, 1e4, 400)
    dc, ec = _peak_offset("sphere", TAU_COLD, T_COLD, 400)
    assert d5 > dc + 0.1, (d5, dc)
    assert abs(dc) < 0.05 + 2 * ec, (dc, ec)


def test_shell_cavity_crossings_terminate():
    """Scattering shell around an empty cavity: photons scattered inwards cross
    the cavity (regression test for the boundary far-root distance) and every
    packet escapes with its weight."""
    n = 400
    geom = dict(kind="shell", r_inner=0.8 * KPC, r_outer=KPC, tau0=2e3, T=1e4,
                v_profile="const_radial", v_max=50 * KMS, step_f=0.05)
    src = dict(kind="point", spectrum="gauss", sigma_v=20 * KMS, seed=12)
    opts = dict(phase="dipole", spectrum=dict(nb=100, lo=-1e8, hi=1e8))
    r = oracle.run(geom, src, opts, 0, n, records=True)
    assert r["stats"]["escaped"] == n and r["stats"]["n_res"] > n
