"""GPU parity of the raytracing driver (Section 3.5) against the oracle.

Projections (FP64 sums of float32 fields) agree with the oracle to 1e-12
relative: only the order of the FP64 additions differs.  Absorption spectra
in FP64 agree to 1e-10 relative (the device Voigt function is within 1e-13
of the oracle's; the rest is summation order).  In mixed precision the Voigt
function and its argument are FP32 (Voigt within 2e-5 relative, argument
rounding a few 1e-7 of x), so tau agrees to 1e-4 relative.

Cases: every axis; ragged grids (no dimension a multiple of 64), rays longer
than one LDS chunk (512 cells), bin counts that leave a partial workgroup,
empty cells (n_HI = 0, some with T = 0), rays split into atomically summed
segments, a call with no rays, and the 512^3 forest workload, checked on
sampled rays of the same launch the benchmark times.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2507_11603_amd import thor  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fields(shape, seed, empty_frac=0.3):
    rng = np.random.default_rng(seed)
    n = (1e-10 * np.exp(rng.normal(0, 1.5, shape))).astype(np.float32)
    T = rng.uniform(5e3, 5e4, shape).astype(np.float32)
    v = rng.normal(0, 3e6, shape).astype(np.float32)
    empty = rng.random(shape) < empty_frac
    n[empty] = 0
    T[empty & (rng.random(shape) < 0.5)] = 0     # T is not used where n_HI = 0
    return n, T, v


@pytest.mark.parametrize("shape", [(37, 45, 70), (600, 3, 5), (2, 3, 5000), (300, 4, 16)])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_projection_matches_oracle(shape, axis, weighted):
    rng = np.random.default_rng(hash((shape, axis, weighted)) % 2 ** 32)
    q = rng.lognormal(0, 2, shape).astype(np.float32)
    w = rng.random(shape, dtype=np.float32) if weighted else None
    ds = 3.1e21
    Qo, Wo = oracle.project(q, w, axis, ds)
    Q, Wd = thor.ray_project(dev(q), None if w is None else dev(w), axis, ds)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Q.cpu().numpy(), Qo, rtol=1e-12)
    np.testing.assert_allclose(Wd.cpu().numpy(), Wo, rtol=1e-12)


FOREST = dict(ds=2.0e22, hubble=6.6e-18, n_sub=3, nb=300, u_lo=-1.5e7, u_hi=2.5e7)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-10), ("mixed", 1e-4)])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_forest_matches_oracle(axis, precision, rtol):
    shape = (11, 13, 70)                          # [z][y][x]
    n, T, v = fields(shape, 100 + axis)
    nj, ni = oracle.ray_image_shape(shape, axis)
    rays = (1, min(3, ni - 1), 2, min(2, nj - 2))
    los = [(i, j) for j in range(rays[2], rays[2] + rays[3]) for i in range(rays[0], rays[0] + rays[1])]
    f = FOREST
    ref = oracle.forest(n, T, v, axis, f["ds"], f["hubble"], f["n_sub"], los, f["nb"], f["u_lo"], f["u_hi"])
    tau = thor.ray_forest(dev(n), dev(T), dev(v), axis, f["ds"], f["hubble"], f["n_sub"], rays,
                          f["nb"], f["u_lo"], f["u_hi"], precision)
    torch.cuda.synchronize()
    got = tau.cpu().numpy().reshape(len(los), f["nb"])
    assert np.all(ref > 0)
    np.testing.assert_allclose(got, ref, rtol=rtol, atol=0)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-10), ("mixed", 1e-4)])
def test_forest_long_ray_spans_lds_chunks(precision, rtol):
    shape = (1, 2, 1100)                          # 1100 cells: three LDS passes
    n, T, v = fields(shape, 7)
    args = dict(ds=1.0e21, hubble=6.6e-18, n_sub=2, nb=257, u_lo=-5e6, u_hi=7.5e7)
    ref = oracle.forest(n, T, v, 0, args["ds"], args["hubble"], args["n_sub"], [(0, 0), (1, 0)],
                        args["nb"], args["u_lo"], args["u_hi"])
    tau = thor.ray_forest(dev(n), dev(T), dev(v), 0, args["ds"], args["hubble"], args["n_sub"],
                          (0, 2, 0, 1), args["nb"], args["u_lo"], args["u_hi"], precision)
    torch.cuda.synchronize()
    np.testing.assert_allclose(tau.cpu().numpy().reshape(2, -1), ref, rtol=rtol)


def test_forest_degenerate_inputs():
    shape = (4, 5, 6)
    n, T, v = fields(shape, 3)
    dn, dT, dv = dev(n), dev(T), dev(v)
    # no rays: an empty result; a caller's output of another shape is refused
    out = torch.empty((1, 0, 8), dtype=torch.float64, device="cuda")
    r = thor.ray_forest(dn, dT, dv, 2, 1e21, 0.0, 1, (0, 0, 0, 1), 8, 0.0, 1e7, out=out)
    torch.cuda.synchronize()
    assert tuple(r.shape) == (1, 0, 8)
    with pytest.raises(ValueError):
        thor.ray_forest(dn, dT, dv, 2, 1e21, 0.0, 1, (0, 0, 0, 1), 8, 0.0, 1e7,
                        out=torch.full((1, 1, 8), 7.0, dtype=torch.float64, device="cuda"))
    # all-empty gas: tau is exactly zero, even where T = 0
    z = torch.zeros_like(dn)
    tau = thor.ray_forest(z, torch.zeros_like(dT), dv, 1, 1e21, 6.6e-18, 2, (0, 6, 0, 4), 40, 0.0, 1e7)
    torch.cuda.synchronize()
    assert torch.count_nonzero(tau).item() == 0
    # one bin, no Hubble flow
    ref = oracle.forest(n, T, v, 2, 1e21, 0.0, 1, [(2, 3)], 1, -1e6, 1e6)
    tau = thor.ray_forest(dn, dT, dv, 2, 1e21, 0.0, 1, (2, 1, 3, 1), 1, -1e6, 1e6)
    torch.cuda.synchronize()
    np.testing.assert_allclose(tau.cpu().numpy().ravel(), ref.ravel(), rtol=1e-10)
    with pytest.raises(thor.ThorError):
        thor.ray_forest(dn, dT, dv, 2, 1e21, 0.0, 1, (5, 2, 0, 1), 8, 0.0, 1e7)


def test_forest_web512_sampled_rays():
    """The 512^3 forest workload (tomography plane j = 256, rays along z),
    launched as the benchmark launches it; a few rays checked against the
    oracle in FP64 and mixed precision."""
    wl = W.forest(512)
    n, T, v = (dev(a) for a in wl["fields"])
    o = wl["opts"]
    picks = [0, 137, 511]
    los = [(o["rays"][0] + p, o["rays"][2]) for p in picks]
    ref = oracle.forest(*wl["fields"], o["axis"], o["ds"], o["hubble"], o["n_sub"], los,
                        o["nb"], o["u_lo"], o["u_hi"])
    for precision, rtol in (("fp64", 1e-10), ("mixed", 1e-4)):
        tau = thor.ray_forest(n, T, v, o["axis"], o["ds"], o["hubble"], o["n_sub"], o["rays"], o["nb"],
                              o["u_lo"], o["u_hi"], precision)
        torch.cuda.synchronize()
        got = tau.cpu().numpy().reshape(-1, o["nb"])
        assert got.shape[0] == 512 and np.all(np.isfinite(got))
        np.testing.assert_allclose(got[picks], ref, rtol=rtol)


def test_projection_web512_column_density():
    """Column-density map of the 512^3 web box along each axis against the
    oracle (whole image)."""
    wl = W.forest(512)
    n = wl["fields"][0]
    dn = dev(n)
    for axis in range(3):
        Q, _ = thor.ray_project(dn, None, axis, wl["opts"]["ds"])
        torch.cuda.synchronize()
        Qo, _ = oracle.project(n, None, axis, wl["opts"]["ds"])
        np.testing.assert_allclose(Q.cpu().numpy(), Qo, rtol=1e-12)


@pytest.mark.parametrize("axis", [0, 2])
def test_projection_unaligned_fields(axis):
    """Fields that start 4 bytes past a 16-byte boundary take the scalar
    loads; the result is the same."""
    shape = (9, 16, 64)
    rng = np.random.default_rng(21)
    q = rng.lognormal(0, 1, shape).astype(np.float32)
    w = rng.random(shape, dtype=np.float32)
    def shifted(a):
        buf = torch.empty(a.size + 1, dtype=torch.float32, device="cuda")
        buf[1:] = torch.from_numpy(a.ravel()).cuda()
        return buf[1:].view(shape)
    Qo, Wo = oracle.project(q, w, axis, 2.0e21)
    Q, Wd = thor.ray_project(shifted(q), shifted(w), axis, 2.0e21)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Q.cpu().numpy(), Qo, rtol=1e-12)
    np.testing.assert_allclose(Wd.cpu().numpy(), Wo, rtol=1e-12)


def test_ray_calls_replay_in_a_graph():
    """Both calls record no memset and allocate nothing once the Dawson tables
    are on the device, so they can be captured: three replays, with eager
    work and synchronisation between them, each equal to the eager result."""
    shape = (300, 4, 16)                          # axis z: a split 16-byte projection
    n, T, v = fields(shape, 9)
    dn, dT, dv = dev(n), dev(T), dev(v)
    Qe, We = thor.ray_project(dn, dT, 2, 1.0e21)
    te = thor.ray_forest(dn, dT, dv, 1, 2.0e21, 6.6e-18, 2, (0, 16, 0, 3), 300, -1e7, 3e7)
    torch.cuda.synchronize()
    Q = torch.zeros_like(Qe); Wd = torch.zeros_like(We); tau = torch.zeros_like(te)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            thor.ray_project(dn, dT, 2, 1.0e21, out=(Q, Wd))
            thor.ray_forest(dn, dT, dv, 1, 2.0e21, 6.6e-18, 2, (0, 16, 0, 3), 300, -1e7, 3e7, out=tau)
    torch.cuda.synchronize()
    for rep in range(3):
        Q.fill_(-1.0); Wd.fill_(-1.0); tau.fill_(-1.0)
        junk = torch.randn(1 << 20, device="cuda").sum()       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        torch.testing.assert_close(Q, Qe, rtol=1e-12, atol=0)
        torch.testing.assert_close(Wd, We, rtol=1e-12, atol=0)
        assert torch.equal(tau, te), rep
