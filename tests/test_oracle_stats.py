"""The chunk two-sample test used for peel cubes (weighted histograms),
checked on the oracle alone: two independent-seed runs of one medium pass,
a changed medium fails."""
import numpy as np
import pytest

import oracle
import workloads as W
from stats_util import chi2_chunks, rebin


def _chunks(wl, n_chunks, per, seed, threads=8):
    """Per chunk: the +z surface-brightness map (cube summed over frequency,
    rebinned to 16^2) and the image-summed peel spectrum (rebinned to 16)."""
    src = dict(wl["src"], seed=seed)
    sb, sp = [], []
    for i in range(n_chunks):
        r = oracle.run_threaded(wl["geom"], src, wl["opts"], i * per, per, threads)
        c = r["cube"][0]
        sb.append(rebin(c.sum(axis=2), (c.shape[0] // 16, c.shape[1] // 16)).ravel())
        sp.append(rebin(c.sum(axis=(0, 1)), (2,)))
    return np.array(sb), np.array(sp)


@pytest.fixture(scope="module")
def shell_pair():
    wl = W.shell(n_grid=32, n_packets=1, cube_nb=64)
    return wl, _chunks(wl, 20, 1500, 11), _chunks(wl, 20, 1500, 12)


def test_chunk_chi2_accepts_independent_runs(shell_pair):
    _, (sb1, sp1), (sb2, sp2) = shell_pair
    for a, b in ((sb1, sb2), (sp1, sp2)):
        chi2, dof, p = chi2_chunks(a, b, 1500, 1500)
        assert dof >= 8
        assert p > 0.001, (chi2, dof, p)


def test_chunk_chi2_rejects_a_changed_medium(shell_pair):
    """An expansion of 150 instead of 200 km/s moves the peel spectrum; an
    albedo of 0 instead of 0.3 dims the map: both are rejected."""
    wl, (sb1, sp1), _ = shell_pair
    g = dict(wl["geom"])
    vx = np.asarray(g["vx"]) * 0.75
    vy = np.asarray(g["vy"]) * 0.75
    vz = np.asarray(g["vz"]) * 0.75
    slow = dict(wl, geom=dict(g, vx=vx, vy=vy, vz=vz))
    _, sp_slow = _chunks(slow, 20, 1500, 13)
    assert chi2_chunks(sp1, sp_slow, 1500, 1500)[2] < 1e-6
    dark = dict(wl, geom=dict(g, albedo=0.0))
    sb_dark, _ = _chunks(dark, 20, 1500, 14)
    assert chi2_chunks(sb1, sb_dark, 1500, 1500)[2] < 1e-6


def test_chunk_chi2_unequal_chunk_sizes():
    """Chunks of very different sizes (the GPU side's are 20x larger): the
    small chunks' pixel sums are strongly skewed, which biases a per-side
    (Welch) variance; the pooled per-packet variance keeps the test
    calibrated on two independent oracle samples of one medium."""
    wl = W.shell(n_grid=64, n_packets=1, cube_nb=64)
    sb_a, sp_a = _chunks(wl, 40, 1000, 21)
    sb_b, sp_b = _chunks(wl, 20, 20000, 22)
    for a, b in ((sb_a, sb_b), (sp_a, sp_b)):
        chi2, dof, p = chi2_chunks(b / 20000, a / 1000, 20000, 1000, min_frac=5e-4)
        assert dof >= 8
        assert p > 0.001, (chi2, dof, p)
