"""Pins of the oracle's building blocks against things other than itself:
published known-answer vectors, an independent Philox implementation,
scipy/mpmath Faddeeva values, closed forms and exact distributions."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ constants
def test_line_constants_literature():
    """Section 2.3.1 definitions evaluated at 1e4 K match the quoted values."""
    want = {}
    for line in open(os.path.join(GOLDEN, "line_constants.txt")):
        if line.strip() and not line.startswith("#"):
            k, v, tol = line.split()
            want[k] = (float(v), float(tol))
    vth, a, s0 = oracle.line_params(1e4)
    for got, key in ((vth, "v_th_cm_s"), (a, "a_voigt"), (s0, "sigma0_cm2")):
        v, tol = want[key]
        assert abs(got / v - 1) < tol, (key, got, v)
    # temperature scalings of the definitions: v_th ~ T^1/2, a and sigma0 ~ T^-1/2
    vth4, a4, s04 = oracle.line_params(4e4)
    assert np.isclose(vth4 / vth, 2.0, rtol=1e-14)
    assert np.isclose(a / a4, 2.0, rtol=1e-14) and np.isclose(s0 / s04, 2.0, rtol=1e-14)


# ------------------------------------------------------------ Voigt
def _grid():
    a = np.logspace(-6, np.log10(5e-2), 23)
    x = np.concatenate([np.linspace(0, 8, 161), np.logspace(np.log10(8.05), 4, 60)])
    return a, x


def test_voigt_vs_scipy_faddeeva():
    """H(a,x) = Re w(x+ia) against scipy.special.wofz (MIT Faddeeva package)."""
    a, x = _grid()
    A, X = np.meshgrid(a, x, indexing="ij")
    got = oracle.voigt(A, X)
    ref = special.wofz(X + 1j * A).real
    rel = np.abs(got - ref) / ref
    assert rel.max() < 1e-12, rel.max()
    # symmetry in x
    assert np.array_equal(oracle.voigt(A[:, :40], -X[:, :40]), got[:, :40])


def test_voigt_vs_mpmath_40_digits():
    import mpmath as mp
    mp.mp.dps = 40
    for a, x in [(1e-6, 0.3), (4.7e-4, 3.2), (4.7e-4, 6.49), (4.7e-4, 6.51), (1.6e-2, 2.0),
                 (5e-2, 5.0), (3e-5, 40.0), (1e-3, 1e3)]:
        z = mp.mpf(x) + 1j * mp.mpf(a)
        ref = float(mp.re(mp.exp(-z * z) * mp.erfc(-1j * z)))
        assert abs(oracle.voigt(a, x) / ref - 1) < 1e-13, (a, x)


def test_voigt_special_cases():
    # H(0, x) = exp(-x^2) (a -> 0 limit, checked at a = 1e-15 where the
    # Lorentzian term is below 1e-12 relative for |x| <= 3)
    x = np.linspace(0, 3, 13)
    assert np.allclose(oracle.voigt(1e-15, x), np.exp(-x * x), rtol=1e-12, atol=0)
    # H(a, 0) = exp(a^2) erfc(a)
    for a in (1e-5, 1e-3, 3e-2):
        assert abs(oracle.voigt(a, 0.0) / (np.exp(a * a) * special.erfc(a)) - 1) < 1e-14
    # far wing: H -> a / (sqrt(pi) x^2) (1 + 3/(2x^2) + 15/(4x^4))
    a, x = 1e-4, 300.0
    asym = a / (np.sqrt(np.pi) * x * x) * (1 + 1.5 / x**2 + 3.75 / x**4)
    assert abs(oracle.voigt(a, x) / asym - 1) < 1e-9
    # normalisation: integral of H over x is sqrt(pi)
    a = 1e-2
    f = lambda t: oracle.lib().or_voigt(a, t)
    tot = 2 * (integrate.quad(f, 0, 6.5, limit=200, epsabs=0, epsrel=1e-12)[0]
               + integrate.quad(f, 6.5, np.inf, limit=200, epsabs=0, epsrel=1e-12)[0])
    assert abs(tot / np.sqrt(np.pi) - 1) < 1e-9


def test_dawson_vs_mpmath():
    import mpmath as mp
    mp.mp.dps = 40
    x = np.linspace(-6.5, 6.5, 131)
    x = x[x != 0]
    ref = np.array([float(mp.sqrt(mp.pi) / 2 * mp.exp(-mp.mpf(v) ** 2) * mp.erfi(mp.mpf(v)))
                    for v in x])
    assert np.abs(oracle.dawson(x) / ref - 1).max() < 1e-15
    assert oracle.dawson([0.0])[0] == 0.0


# ------------------------------------------------------------ x_cw (Appendix A.2)
def test_lambert_wm1_vs_mpmath():
    """The lower branch of Lambert's W against mpmath at 40 digits, from
    z -> 0- to the branch point -1/e (where W is ill-conditioned: there the
    bound is the conditioning, |dW/dz| ~ 1/sqrt(2 e (z + 1/e)))."""
    import mpmath as mp
    mp.mp.dps = 40
    z = -np.concatenate([np.logspace(-300, -1, 120), np.linspace(0.1, 1 / np.e, 60)[1:-1],
                         [1 / np.e - 1e-6, 1 / np.e - 1e-12]])
    got = oracle.lambert_wm1(z)
    ref = np.array([float(mp.lambertw(mp.mpf(v), -1)) for v in z])
    far = np.abs(1 + ref) > 1e-2
    assert np.abs(got[far] / ref[far] - 1).max() < 1e-14
    assert np.abs(got[~far] - ref[~far]).max() < 1e-7
    assert np.isnan(oracle.lambert_wm1([-0.5, 0.0, 0.1])).all()


def test_xcw_exact_is_the_core_wing_crossing():
    """x_cw solves exp(-x^2) = a/(sqrt(pi) x^2) and equals
    sqrt(-W_{-1}(-a/sqrt(pi))) by scipy's Lambert W; it lies beyond the
    inflexion of the core (x > 1) and grows as a falls."""
    a = np.logspace(-8, -1, 120)
    x = oracle.xcw(a)
    assert np.abs(np.exp(-x ** 2) * np.sqrt(np.pi) * x ** 2 / a - 1).max() < 1e-12
    ref = np.sqrt(-special.lambertw(-a / np.sqrt(np.pi), -1).real)
    assert np.abs(x / ref - 1).max() < 1e-14
    assert np.all(np.diff(x) < 0) and x.min() > 1.0
    # at 1e4 K (a = 4.72e-4) the core turns into the wing near 3.25 Doppler widths
    _, a4, _ = oracle.line_params(1e4)
    assert abs(oracle.xcw([a4])[0] - 3.2544) < 1e-3


def test_xcw_b25_within_its_stated_accuracy():
    """The Appendix A.2 quartic in ln a stays within 0.6 % of the exact x_cw
    over the Lyman-alpha temperature range (a from 1.5e-5 to 1e-2, about
    T = 22 K to 1e7 K) and departs from it outside (it is a fit, not a
    limit: 10 % at a = 1e-6)."""
    a = np.logspace(np.log10(1.5e-5), -2, 500)
    rel = np.abs(oracle.xcw(a, "b25") / oracle.xcw(a) - 1)
    assert rel.max() < 6e-3, rel.max()
    assert abs(oracle.xcw([1e-6], "b25")[0] / oracle.xcw([1e-6])[0] - 1) > 0.05


# ------------------------------------------------------------ Philox
def _kat_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_published_kat():
    for ctr, key, out in _kat_rows():
        assert oracle.philox(ctr, key) == out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_vs_rocrand_header(tmp_path):
    """Random counters/keys against AMD rocRAND's independent implementation."""
    exe = tmp_path / "kat"
    subprocess.check_call(["hipcc", "-O1", "-o", str(exe),
                           os.path.join(GOLDEN, "philox_rocrand_kat.cpp")], cwd=str(tmp_path))
    rng = np.random.default_rng(11)
    cases = rng.integers(0, 2**32, size=(64, 6), dtype=np.uint64)
    inp = "\n".join(" ".join("%08x" % v for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    for row, line in zip(cases, out.strip().splitlines()):
        want = [int(t, 16) for t in line.split()]
        assert oracle.philox(row[:4], row[4:]) == want


def test_draw_uniform_mapping():
    """Two 53-bit uniforms per call, from (w0,w1) and (w2,w3)."""
    w = oracle.philox([3, 4, 5, 6], [1, 2])
    ua, ub = oracle.draw(1, 2, 3, 4, 5 | (6 << 32))
    assert ua == (((w[0] << 32) | w[1]) >> 11) * 2.0**-53
    assert ub == (((w[2] << 32) | w[3]) >> 11) * 2.0**-53
    u = np.array([oracle.draw(9, 0, 0, 1, i)[0] for i in range(20000)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# ------------------------------------------------------------ u_parallel
def _upar_mass(lo, hi, x, a):
    """Integral of exp(-u^2)/((x-u)^2+a^2) over [lo, hi]: in u near the
    Lorentzian spike via u = x + a tan(theta) (du/((x-u)^2+a^2) = dtheta/a),
    elsewhere directly in u."""
    W = 100.0 * a
    g = lambda u: np.exp(-u * u) / ((x - u) ** 2 + a * a)
    gt = lambda th: np.exp(-(x + a * np.tan(th)) ** 2) / a
    tot = 0.0
    for (p, q, spike) in ((-np.inf, x - W, False), (x - W, x + W, True), (x + W, np.inf, False)):
        p2, q2 = max(p, lo), min(q, hi)
        if q2 <= p2:
            continue
        if spike:
            tot += integrate.quad(gt, np.arctan((p2 - x) / a), np.arctan((q2 - x) / a),
                                  limit=200, epsabs=0, epsrel=1e-11)[0]
        else:
            pts = [v for v in (-1.0, 0.0, 1.0) if p2 < v < q2]
            if np.isinf(p2) or np.isinf(q2):
                tot += integrate.quad(g, p2, q2, limit=400, epsabs=0, epsrel=1e-11)[0]
            else:
                tot += integrate.quad(g, p2, q2, points=pts or None, limit=400, epsabs=0,
                                      epsrel=1e-11)[0]
    return tot


def _upar_cdf_at(edges, x, a):
    norm = np.pi * special.wofz(x + 1j * a).real / a
    return np.array([_upar_mass(-np.inf, e, x, a) for e in edges]) / norm


@pytest.mark.parametrize("a", [1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("x", [0.0, 0.5, 1.5, 2.2, 2.3, 3.0, 5.0, 10.0, 40.0])
def test_upar_distribution(x, a):
    """Samples follow eq. (uparallel) exactly: binned chi^2 and a KS bound on
    edges spanning the Gaussian bulk and the Lorentzian spike at u = x."""
    n = 20000
    u, tr = oracle.sample_upar(x, a, n, seed=101)
    edges = np.unique(np.concatenate([np.linspace(-3.5, 3.5, 57),
                                      x + a * np.tan(np.linspace(-1.45, 1.45, 31))]))
    edges = edges[(edges > -11) & (edges < 11.5)]
    cdf = _upar_cdf_at(edges, x, a)
    emp = np.searchsorted(np.sort(u), edges, side="right") / n
    d = np.abs(emp - cdf).max()
    assert d < 1.95 / np.sqrt(n), d       # KS critical value at ~0.1 %
    # chi^2 on the cells between edges (merged to >= 20 expected)
    probs = np.diff(np.concatenate([[0.0], cdf, [1.0]]))
    counts = np.diff(np.concatenate([[0], np.searchsorted(np.sort(u), edges, side="right"), [n]]))
    exp_c, obs_c, acc_e, acc_o = [], [], 0.0, 0
    for p_, c_ in zip(probs, counts):
        acc_e += p_ * n
        acc_o += c_
        if acc_e >= 20:
            exp_c.append(acc_e); obs_c.append(acc_o); acc_e, acc_o = 0.0, 0
    exp_c[-1] += acc_e; obs_c[-1] += acc_o
    chi2 = np.sum((np.array(obs_c) - np.array(exp_c)) ** 2 / np.array(exp_c))
    assert stats.chi2.sf(chi2, len(exp_c) - 1) > 1e-4
    # closed-form moments: E[x - u] = a L / H, E[(x-u)^2] = a/(sqrt(pi) H) - a^2
    w = special.wofz(x + 1j * a)
    m1 = a * w.imag / w.real
    s = x - u
    assert abs(s.mean() - m1) < 5 * s.std() / np.sqrt(n) + 1e-12
    m2 = a / (np.sqrt(np.pi) * w.real) - a * a
    assert abs(np.mean(s * s) - m2) < 5 * np.std(s * s) / np.sqrt(n) + 1e-12
    # expected trials = envelope mass / target mass
    et = oracle.upar_expected_trials(x, a)
    assert abs(tr.mean() - et) < 5 * np.sqrt(max(et * (et - 1), 1e-3) / n) + 1e-9


def test_upar_sign_symmetry():
    u1, _ = oracle.sample_upar(3.0, 1e-3, 500, seed=5)
    u2, _ = oracle.sample_upar(-3.0, 1e-3, 500, seed=5)
    assert np.array_equal(u1, -u2)


# ------------------------------------------------------------ phase functions
@pytest.mark.parametrize("phase,cdf,m2", [
    ("iso", lambda m: (m + 1) / 2, 1 / 3),
    ("dipole", lambda m: 0.375 * (m + m**3 / 3) + 0.5, 2 / 5),
    ("core_wing", lambda m: (11 * m + m**3) / 24 + 0.5, 16 / 45),
])
def test_phase_samplers(phase, cdf, m2):
    U = np.random.default_rng(3).random(40000)
    mu = oracle.sample_mu(phase, U)
    assert np.all(np.abs(mu) <= 1 + 1e-15)
    assert np.allclose(cdf(mu), U, atol=1e-13)          # exact inverse of the CDF
    assert abs(np.mean(mu**2) - m2) < 5 * np.std(mu**2) / 200


def test_hg_sampler():
    g = 0.73
    U = np.random.default_rng(4).random(40000)
    mu = oracle.sample_mu("hg", U, g)
    cdf = lambda m: (1 - g * g) / (2 * g) * (1 / np.sqrt(1 + g * g - 2 * g * m) - 1 / (1 + g))
    assert np.allclose(cdf(mu), U, atol=1e-12)
    assert abs(mu.mean() - g) < 5 * mu.std() / 200


def test_basis_orthonormal():
    rng = np.random.default_rng(8)
    v = rng.normal(size=(500, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    v = np.vstack([v, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1e-9, -1]]])
    v /= np.linalg.norm(v, axis=1)[:, None]
    for n in v:
        e1, e2 = oracle.basis(n)
        M = np.array([n, e1, e2])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-13)
