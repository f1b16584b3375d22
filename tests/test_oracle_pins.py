"""Pins of the oracle's generator and of its single-scattering step against
what the paper and the mathematics fix, independently of the oracle's own
formulas: brute-force sampling, closed-form moments of the redistribution
(via the Faddeeva function), exact emission probabilities computed here, and
the frame invariance of a uniformly moving medium.

Sections cited: 2.1 and 3.4 "Emission" (n_HI^2-weighted cells, thermal
profile in the gas frame), 2.3.1 (eqs. uperp, uparallel and
doublelorentztransform), 3.4.2 (core skipping)."""
import numpy as np
import pytest
from scipy import special, stats

import oracle
import workloads as W

KPC, KMS = W.KPC, W.KMS
M2 = {"iso": 1.0 / 3.0, "dipole": 2.0 / 5.0}      # E[mu^2] of the phase functions


# ------------------------------------------------------------ core skipping
def test_core_skip_truncation_matches_brute_force():
    """Section 3.4.2 (read as a 2D radial truncation): below x_crit the
    perpendicular atom velocity is the Gaussian of eq. uperp conditioned on
    |u_perp| > x_crit.  Brute force: numpy normals of variance 1/2 per
    component, kept when their radius exceeds x_crit; two-sample KS on the
    radius and on one component."""
    xc, n = 1.2, 40000
    s = oracle.scatter_resonant(0.7, 1e-3, (0.3, -0.4, np.sqrt(0.75)), n, x_crit=xc)
    rho = np.hypot(s["uperp"][:, 0], s["uperp"][:, 1])
    rng = np.random.default_rng(77)
    g = rng.normal(scale=np.sqrt(0.5), size=(6 * n, 2))
    g = g[np.hypot(g[:, 0], g[:, 1]) > xc][:n]
    assert len(g) == n
    assert stats.ks_2samp(rho, np.hypot(g[:, 0], g[:, 1])).pvalue > 1e-3
    assert stats.ks_2samp(s["uperp"][:, 0], g[:, 0]).pvalue > 1e-3
    assert rho.min() > xc


def test_core_skip_closed_form_and_threshold():
    """Truncated at x_crit = 3 (the web box's value): rho^2 - x_crit^2 ~ Exp(1)
    (the radial density of a 2D Gaussian of variance 1/2 per component is
    2 rho exp(-rho^2), memoryless in rho^2).  At |x| >= x_crit there is no
    truncation: each component is N(0, 1/2)."""
    n = 40000
    k = (0.0, 0.6, 0.8)
    s = oracle.scatter_resonant(-2.5, 4.7e-4, k, n, x_crit=3.0)
    r2 = np.sum(s["uperp"] ** 2, axis=1)
    assert stats.kstest(r2 - 9.0, "expon").pvalue > 1e-3
    s = oracle.scatter_resonant(3.5, 4.7e-4, k, n, x_crit=3.0)
    for j in range(2):
        assert stats.kstest(s["uperp"][:, j], "norm", args=(0.0, np.sqrt(0.5))).pvalue > 1e-3


# --------------------------------------------------------- redistribution
def _moments(x, a, m2, rho2):
    """E[x_out] and E[x_out^2] for a phase function with E[mu] = 0 and
    E[mu^2] = m2 (independent of the atom), with E|u_perp|^2 = rho2.
    From w = H + iL at x + ia: E[x - u_par] = a L / H, E[(x - u_par)^2] =
    a / (sqrt(pi) H) - a^2; x_out = (x - u_par) + u.k_out with
    u.k_out = u_par mu + sqrt(1 - mu^2) u_perp.(cos phi, sin phi)."""
    w = special.wofz(x + 1j * a)
    e1 = a * w.imag / w.real
    e2 = a / (np.sqrt(np.pi) * w.real) - a * a
    upar2 = x * x - 2.0 * x * e1 + e2
    return e1, e2 + m2 * upar2 + (1.0 - m2) * rho2 / 2.0


@pytest.mark.parametrize("x,a,phase,xc", [
    (0.0, 1e-3, "iso", 0.0), (1.5, 1e-3, "dipole", 0.0), (3.5, 4.7e-4, "dipole", 0.0),
    (8.0, 1e-2, "iso", 0.0), (-2.2, 4.7e-4, "dipole", 0.0), (1.0, 2e-3, "dipole", 3.0),
    (2.7, 1.5e-2, "iso", 0.0)])
def test_redistribution_moments(x, a, phase, xc):
    """Eq. doublelorentztransform without recoil, P5: for a phase function
    symmetric in mu, E[x_out | x] = a L(a,x) / H(a,x), and the second moment
    follows from the u_par moments and E[mu^2] (1/3 isotropic, 2/5 dipole).
    Also the outgoing directions: unit length, E[mu_out] = 0, E[mu_out^2] =
    E[mu^2] relative to the incoming direction."""
    n = 200000
    k = np.array([0.48, -0.6, 0.64])
    s = oracle.scatter_resonant(x, a, k, n, x_crit=xc, phase=phase, seed=31)
    rho2 = 1.0 + (xc * xc if abs(x) < xc else 0.0)
    e1, e2 = _moments(x, a, M2[phase], rho2)
    xo = s["x_out"]
    assert abs(xo.mean() - e1) < 4 * xo.std() / np.sqrt(n)
    assert abs(np.mean(xo * xo) - e2) < 4 * np.std(xo * xo) / np.sqrt(n)
    ko = s["kout"]
    assert np.allclose(np.linalg.norm(ko, axis=1), 1.0, atol=1e-12)
    mu = ko @ k
    assert abs(mu.mean()) < 4 * mu.std() / np.sqrt(n)
    assert abs(np.mean(mu * mu) - M2[phase]) < 4 * np.std(mu * mu) / np.sqrt(n)
    # x_out = x_atom + u.k_out with u = u_par k + u_perp in the plane of k:
    # E[(x_out - x_atom) mu] = E[u_par] E[mu^2] (a forward scattering keeps the
    # lab-frame frequency, a backward one reflects u_par)
    assert np.allclose(s["x_atom"], x - s["upar"], rtol=0, atol=1e-12 * (1 + abs(x)))
    c = (xo - s["x_atom"]) * mu
    assert abs(c.mean() - (x - e1) * M2[phase]) < 4 * c.std() / np.sqrt(n)


def test_core_wing_mean_redistribution():
    """The core/wing mix (Section 2.3.1) picks its phase function by the atom
    frame frequency, but both choices are symmetric in mu, so E[x_out | x] =
    a L / H still holds; the core form is used exactly when |x - u_par| < 0.2."""
    n = 200000
    x, a = 3.0, 1e-3      # about two thirds of the atoms resonant (core), one third wing
    s = oracle.scatter_resonant(x, a, (0.0, 0.0, 1.0), n, phase="core_wing", seed=5)
    e1, _ = _moments(x, a, 0.4, 1.0)
    assert abs(s["x_out"].mean() - e1) < 4 * s["x_out"].std() / np.sqrt(n)
    core = np.abs(s["x_atom"]) < 0.2
    assert np.array_equal(s["phase"] == 2, core) and 0.3 < core.mean() < 0.9


# --------------------------------------------------------------- emission
def _small_grid(rng, shape=(4, 5, 6), zeros=True):
    nz, ny, nx = shape
    n = rng.lognormal(-11.0, 1.0, size=shape).astype(np.float32)
    if zeros:
        n[rng.random(shape) < 0.2] = 0.0
    T = rng.uniform(3e3, 3e4, size=shape).astype(np.float32)
    v = [rng.normal(0.0, 80 * KMS, size=shape).astype(np.float32) for _ in range(3)]
    L = 2.0 * KPC
    geom = dict(kind="grid", lo=(-KPC, -0.5 * KPC, 0.0), hi=(KPC, 1.5 * KPC, L),
                n_HI_field=n, T_field=T, vx=v[0], vy=v[1], vz=v[2])
    return geom, n, T, v


def test_emission_cells_follow_n_squared():
    """Section 3.4 "Emission" with an n_HI^2 emissivity (recombination): cell c
    is drawn with probability n_c^2 / sum n^2 (computed here), and the packet
    starts at a uniform point inside it."""
    rng = np.random.default_rng(2024)
    geom, n, _, _ = _small_grid(rng)
    N = 200000
    e = oracle.emit(geom, dict(kind="cell_n2", spectrum="delta", seed=4), 0, N)
    nz, ny, nx = n.shape
    flat = (e["cell"][:, 2] * ny + e["cell"][:, 1]) * nx + e["cell"][:, 0]
    counts = np.bincount(flat, minlength=n.size)
    p = (n.astype(np.float64) ** 2).ravel()
    p /= p.sum()
    assert np.all(counts[p == 0] == 0)
    keep = p > 0
    chi2 = np.sum((counts[keep] - N * p[keep]) ** 2 / (N * p[keep]))
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3
    lo = np.array(geom["lo"])
    dx = (np.array(geom["hi"]) - lo) / np.array([nx, ny, nz])
    frac = (e["pos"] - lo) / dx - e["cell"]
    for j in range(3):
        assert np.all((frac[:, j] >= 0) & (frac[:, j] < 1 + 1e-9))
        assert stats.kstest(frac[:, j], "uniform").pvalue > 1e-3
    # isotropic directions: mu uniform on [-1, 1], azimuth uniform
    d = e["dir"]
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    assert stats.kstest((d[:, 2] + 1) / 2, "uniform").pvalue > 1e-3
    phi = (np.arctan2(d[:, 1], d[:, 0]) / (2 * np.pi)) % 1.0
    assert stats.kstest(phi, "uniform").pvalue > 1e-3


def test_emission_thermal_profile_in_gas_frame():
    """Thermal emission (Section 2.1: the intrinsic line of the emitting gas),
    shifted to the lab frame by the cell velocity (Section 3.4): gas-frame
    offsets are N(dv0, v_th/sqrt 2) with v_th = sqrt(2kT/m_H) of the cell, and
    lab dv - gas dv = v_cell . k."""
    rng = np.random.default_rng(7)
    geom, n, T, v = _small_grid(rng, zeros=False)
    N, dv0 = 100000, 35 * KMS
    e = oracle.emit(geom, dict(kind="cell_n2", spectrum="thermal", dv0=dv0, seed=9), 0, N)
    cz, cy, cx = e["cell"][:, 2], e["cell"][:, 1], e["cell"][:, 0]
    vth = np.array([oracle.line_params(t)[0] for t in T[cz, cy, cx]])
    z = (e["dv_loc"] - dv0) / (vth / np.sqrt(2.0))
    assert stats.kstest(z, "norm").pvalue > 1e-3
    vk = sum(v[j][cz, cy, cx].astype(np.float64) * e["dir"][:, j] for j in range(3))
    assert np.allclose(e["dv"] - e["dv_loc"], vk, rtol=0, atol=1e-6 * 80 * KMS)


def test_emission_gaussian_source_and_point():
    """A point source with a Gaussian line: every packet at the source point,
    dv ~ N(dv0, sigma_v), and no gas-frame shift applied."""
    geom = dict(kind="shell", r_inner=0.0, r_outer=KPC, tau0=1e4, T=1e4)
    src = dict(kind="point", pos=(0.1 * KPC, -0.2 * KPC, 0.0), spectrum="gauss", dv0=-10 * KMS,
               sigma_v=20 * KMS, seed=3)
    e = oracle.emit(geom, src, 0, 50000)
    assert np.all(e["pos"] == np.array(src["pos"]))
    assert stats.kstest((e["dv"] + 10 * KMS) / (20 * KMS), "norm").pvalue > 1e-3
    assert np.all(e["dv_loc"] == 0.0)


# ----------------------------------------------------------- moving medium
def test_uniformly_moving_grid_is_the_static_one_shifted():
    """Galilean invariance of the gas-frame physics (Section 2.2: the cross
    section is evaluated in the local fluid frame; Section 3.4 "Emission": the
    thermal line is shifted to the lab frame by v.k).  A homogeneous grid
    moving with V along +z scatters every packet as the static grid does (the
    same random draws meet the same gas-frame frequencies), and the peel-off
    spectrum towards observer k_o is the static one shifted by V.k_o: by +V for
    +z, by -V for -z, unshifted for +x."""
    nc, N = 8, 1500
    V, wbin = 100 * KMS, 10 * KMS
    shape = (nc, nc, nc)
    dens = np.full(shape, 2e-7, np.float32)          # line-centre tau of ~ 4e3 per cell
    temp = np.full(shape, 1e4, np.float32)
    zero = np.zeros(shape, np.float32)
    cube = dict(nx=4, ny=4, nb=160, img_lo=(0.0, 0.0), img_hi=(KPC, KPC), v_lo=-800 * KMS, v_hi=800 * KMS)
    opts = dict(phase="dipole", observers=["+z", "-z", "+x"], cube=cube,
                spectrum=dict(nb=10, lo=-800 * KMS, hi=800 * KMS), tau_cut=40.0)
    src = dict(kind="cell_n2", spectrum="thermal", seed=13)
    out = []
    for vz in (zero, np.full(shape, V, np.float32)):
        geom = dict(kind="grid", lo=(0.0, 0.0, 0.0), hi=(KPC, KPC, KPC), n_HI_field=dens, T_field=temp,
                    vx=zero, vy=zero, vz=vz)
        out.append(oracle.run_parallel(geom, src, opts, 0, N, records=True))
    st, mv = out
    same = np.mean(st["records"]["n_res"] == mv["records"]["n_res"])
    assert same > 0.99, same
    assert st["stats"]["n_res"] > 10 * N
    sh = int(round(V / wbin))
    spec_s = st["cube"].sum(axis=(1, 2))        # [observer][bin]
    spec_m = mv["cube"].sum(axis=(1, 2))
    tot = spec_s.sum(axis=1)
    for o, shift in ((0, sh), (1, -sh), (2, 0)):
        moved = np.roll(spec_m[o], -shift)
        assert np.max(np.abs(moved - spec_s[o])) < 0.01 * tot[o], o
        assert abs(spec_m[o].sum() - tot[o]) < 0.005 * tot[o]
    # and it is a shift, not the same spectrum: the +z observer's mean moves by V
    vc = cube["v_lo"] + (np.arange(cube["nb"]) + 0.5) * wbin
    mean = lambda s: np.sum(s * vc) / s.sum()
    assert abs(mean(spec_m[0]) - mean(spec_s[0]) - V) < 0.02 * V
    assert abs(mean(spec_m[2]) - mean(spec_s[2])) < 0.02 * V
