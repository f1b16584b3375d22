"""Pins of the raytracing oracle (Section 3.5): projections and Lyman-alpha
absorption spectra, against closed forms and invariants that do not come from
the oracle's own formulas.

* Projection: a uniform field gives n L; a field linear in the ray coordinate
  gives an arithmetic series; a field projected along one axis equals the
  transposed field projected along another (catches index and transposition
  mistakes); the w-weighted mean of a constant is that constant.
* Absorption (eq. abs): the Gunn-Peterson optical depth of a uniform expanding
  medium, tau = pi e^2 f lambda n / (m_e c H), for two temperatures (the
  plateau does not depend on T); the equivalent width of one optically thin
  absorber, int tau du = N pi e^2 f lambda / (m_e c); the Lorentz wing
  N sigma0 a / (sqrt(pi) x^2) far from the line; the line centre at
  u = v + H s (signs of both velocity terms); and the same spectrum for the
  same ray along any axis.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

# physical constants (cgs) for the closed forms
E_CHARGE = 4.80320471e-10
M_E = 9.1093837015e-28
C_LIGHT = 2.99792458e10
F12 = 0.4162
LAMBDA = 1215.67e-8
A21 = 6.265e8
K_B = 1.380649e-16
M_H = 1.6735575e-24
SIGMA_VTH = np.pi * E_CHARGE ** 2 * F12 * LAMBDA / (M_E * C_LIGHT)   # sigma0 v_th sqrt(pi)


def vth_of(T):
    return np.sqrt(2 * K_B * T / M_H)


# ----------------------------------------------------------------- projection
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_projection_uniform_and_linear(axis):
    shape = (5, 6, 7)                               # [z][y][x]
    n_ray = shape[2 - axis]
    ds = 3.0e20
    Q, W = oracle.project(np.full(shape, 2.5, np.float32), None, axis, ds)
    assert Q.shape == oracle.ray_image_shape(shape, axis)
    np.testing.assert_allclose(Q, 2.5 * n_ray * ds, rtol=1e-15)
    np.testing.assert_allclose(W, n_ray * ds, rtol=1e-15)
    # q = k (cell index along the ray): Q = ds n (n - 1) / 2
    k = np.arange(n_ray, dtype=np.float32)
    q = np.broadcast_to(k.reshape([-1 if d == 2 - axis else 1 for d in range(3)]), shape)
    Q, _ = oracle.project(q, None, axis, ds)
    np.testing.assert_allclose(Q, ds * n_ray * (n_ray - 1) / 2, rtol=1e-15)


def test_projection_axes_agree_on_transposed_fields():
    rng = np.random.default_rng(5)
    f = rng.random((4, 5, 6), dtype=np.float32)
    w = rng.random((4, 5, 6), dtype=np.float32)
    Qz, Wz = oracle.project(f, w, 2, 1.5)
    # swap x and z: rays along the new x are the old rays along z, and the new
    # (y, z) image index is the old (y, x)
    ft, wt = np.ascontiguousarray(f.transpose(2, 1, 0)), np.ascontiguousarray(w.transpose(2, 1, 0))
    Qx, Wx = oracle.project(ft, wt, 0, 1.5)
    np.testing.assert_allclose(Qx.T, Qz, rtol=1e-13)
    np.testing.assert_allclose(Wx.T, Wz, rtol=1e-13)
    # the weighted mean of a constant field is that constant
    Qc, Wc = oracle.project(np.full_like(f, 7.0), w, 1, 1.5)
    np.testing.assert_allclose(Qc / Wc, 7.0, rtol=1e-13)


def test_projection_rejects_bad_axis():
    with pytest.raises(ValueError):
        oracle.project(np.ones((2, 2, 2), np.float32), None, 3, 1.0)


# ------------------------------------------------------------------ forest
@pytest.mark.parametrize("T", [1e4, 4e4])
def test_gunn_peterson_plateau(T):
    """Uniform n_HI, no peculiar velocity, Hubble rate H: far from the ends of
    the ray, tau = pi e^2 f lambda n / (m_e c H), independent of T."""
    n_hi, H, n_cells, n_sub = 1e-11, 1e-17, 400, 4
    vth = vth_of(1e4)
    ds = vth / 8 / H                                 # H ds = v_th(1e4) / 8
    shape = (1, 1, n_cells)
    tau = oracle.forest(np.full(shape, n_hi, np.float32), np.full(shape, T, np.float32),
                        np.zeros(shape, np.float32), 0, ds, H, n_sub, [[0, 0]], 24,
                        0.35 * H * n_cells * ds, 0.65 * H * n_cells * ds)
    gp = SIGMA_VTH * n_hi / H
    np.testing.assert_allclose(tau[0], gp, rtol=1e-4)


def test_thin_absorber_equivalent_width_wing_and_centre():
    """One cell of column N and peculiar velocity v, no Hubble flow: the
    spectrum integrates to N pi e^2 f lambda / (m_e c), peaks at u = v, and
    falls as N sigma0 a / (sqrt(pi) x^2) in the damping wing."""
    T, v, ds, n_hi = 1e4, 3.0e6, 1e18, 1e-2      # N = 1e16 cm^-2 (optically thin)
    vth = vth_of(T)
    a = A21 * LAMBDA / (4 * np.pi * vth)
    shape = (3, 1, 1)
    nf = np.zeros(shape, np.float32)
    nf[1] = n_hi
    vf = np.full(shape, v, np.float32)
    nb, half = 8000, 400 * vth
    tau = oracle.forest(nf, np.full(shape, T, np.float32), vf, 2, ds, 0.0, 2, [[0, 0]], nb,
                        float(np.float32(v)) - half, float(np.float32(v)) + half)[0]
    du = 2 * half / nb
    N = n_hi * ds
    # beyond +-400 v_th the Lorentz wing holds 2 a / (pi 400) of the sqrt(pi) total
    ew = tau.sum() * du / (1 - 2 * a / (np.pi * 400) / np.sqrt(np.pi))
    np.testing.assert_allclose(ew, N * SIGMA_VTH, rtol=1e-4)
    assert abs(np.argmax(tau) - nb // 2) <= 1       # centre at u = v (bins straddle it)
    u = float(np.float32(v)) - half + (np.arange(nb) + 0.5) * du
    x = (u - float(np.float32(v))) / vth
    sigma0 = SIGMA_VTH / (vth * np.sqrt(np.pi))
    far = np.abs(x) > 100
    wing = N * sigma0 * a / (np.sqrt(np.pi) * x[far] ** 2) * (1 + 1.5 / x[far] ** 2)
    np.testing.assert_allclose(tau[far], wing, rtol=1e-4)


def test_hubble_shift_places_absorber():
    """An absorber in cell k with v = 0 and Hubble rate H absorbs at
    u = H (k + 1/2) ds (one sub-step per cell)."""
    T, H, n_cells, k = 2e4, 1e-17, 64, 41
    vth = vth_of(T)
    ds = vth / H                                     # one v_th per cell
    shape = (1, n_cells, 1)
    nf = np.zeros(shape, np.float32)
    nf[0, k, 0] = 1e-9
    nb = 64 * 20
    tau = oracle.forest(nf, np.full(shape, T, np.float32), np.zeros(shape, np.float32), 1, ds,
                        H, 1, [[0, 0]], nb, 0.0, n_cells * vth)[0]
    du = n_cells * vth / nb
    u_peak = (np.argmax(tau) + 0.5) * du
    assert abs(u_peak - H * (k + 0.5) * ds) <= du


def test_forest_same_ray_along_every_axis():
    rng = np.random.default_rng(11)
    n = 24
    nh = (10 ** rng.uniform(-12, -8, n)).astype(np.float32)
    T = rng.uniform(5e3, 3e4, n).astype(np.float32)
    v = rng.normal(0, 2e6, n).astype(np.float32)
    args = dict(ds=2e21, hubble=1e-17, n_sub=3, nb=90, u_lo=-2e6, u_hi=6e6)
    taus = []
    for axis in range(3):
        shape = [1, 1, 1]
        shape[2 - axis] = n
        taus.append(oracle.forest(nh.reshape(shape), T.reshape(shape), v.reshape(shape), axis,
                                  args["ds"], args["hubble"], args["n_sub"], [[0, 0]],
                                  args["nb"], args["u_lo"], args["u_hi"])[0])
    np.testing.assert_allclose(taus[1], taus[0], rtol=1e-14)
    np.testing.assert_allclose(taus[2], taus[0], rtol=1e-14)
    assert np.all(taus[0] > 0)


def test_forest_rejects_bad_rays():
    f = np.ones((2, 2, 2), np.float32)
    with pytest.raises(ValueError):
        oracle.forest(f, f, f, 2, 1.0, 0.0, 1, [[2, 0]], 4, 0.0, 1.0)
    with pytest.raises(ValueError):
        oracle.forest(f, f, f, 2, 1.0, 0.0, 0, [[0, 0]], 4, 0.0, 1.0)


def _wing_series(a, x, n_terms):
    """Asymptotic series of w(z) at z = x + i a, sum_n (2n-1)!!/2^n z^-(2n+1),
    through n = n_terms; H = Re w."""
    z = complex(x, a)
    term, total = 1.0 / z, 0.0
    for n in range(n_terms + 1):
        total += term
        term *= (2 * n + 1) / (2 * z * z)
    return (1j / np.sqrt(np.pi) * total).real


@pytest.mark.parametrize("a", [1e-4, 5e-4, 1.3e-2, 0.05])
def test_far_wing_series_lengths(a):
    """The absorption-spectrum kernels evaluate H(a, x) far from the line by
    the asymptotic series of w(z): FP64 with 4 terms from |x| = 40, 6 from
    |x| = 20 and 9 from |x| = 12, FP32 with 4 terms from |x| = 6.5.  At and
    beyond those thresholds the truncated series stays within 3.5e-14 (FP64)
    and 3e-6 (FP32) of the oracle's Voigt function, for damping parameters of
    10 K to 1e6 K gas."""
    for x0, n, tol in ((40.0, 4, 3.5e-14), (20.0, 6, 1.1e-14), (12.0, 9, 1.1e-14), (6.5, 4, 3e-6)):
        for x in (x0, x0 * 1.5, x0 * 4, -x0):
            h = oracle.voigt(a, x)
            assert abs(_wing_series(a, x, n) / h - 1) < tol, (x0, n, x)
