"""Statistical comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np
from scipy import stats


def chi2_two_sample(h1, h2, min_count=10.0):
    """Two-sample chi^2 homogeneity test of two histograms of counts (equal
    or unequal totals), merging adjacent bins until n1 + n2 >= min_count.
    Returns (statistic, dof, p-value)."""
    h1 = np.asarray(h1, float)
    h2 = np.asarray(h2, float)
    N1, N2 = h1.sum(), h2.sum()
    a, b, m1, m2 = [], [], 0.0, 0.0
    for x, y in zip(h1, h2):
        m1 += x; m2 += y
        if m1 + m2 >= min_count:
            a.append(m1); b.append(m2); m1 = m2 = 0.0
    if a and (m1 + m2) > 0:
        a[-1] += m1; b[-1] += m2
    a, b = np.array(a), np.array(b)
    k1, k2 = np.sqrt(N2 / N1), np.sqrt(N1 / N2)
    chi2 = np.sum((k1 * a - k2 * b) ** 2 / (a + b))
    dof = len(a) - 1
    return chi2, dof, stats.chi2.sf(chi2, dof)


def chi2_weighted(w1, s1, w2, s2, min_rel=0.2):
    """Weighted two-sample chi^2 (Gagunashvili 2006) of two normalised weighted
    histograms: w = sum of weights per bin, s = sum of squared weights per bin.
    Bins where either side's relative error exceeds min_rel... are merged."""
    w1, s1, w2, s2 = map(lambda v: np.asarray(v, float), (w1, s1, w2, s2))
    W1, W2 = w1.sum(), w2.sum()
    keep = (s1 > 0) & (s2 > 0) & (w1 > 0) & (w2 > 0)
    keep &= (np.sqrt(s1) / np.maximum(w1, 1e-300) < min_rel) & (np.sqrt(s2) / np.maximum(w2, 1e-300) < min_rel)
    w1, s1, w2, s2 = w1[keep], s1[keep], w2[keep], s2[keep]
    num = (W1 * w2 - W2 * w1) ** 2
    den = W1 ** 2 * s2 + W2 ** 2 * s1
    chi2 = np.sum(num / den)
    dof = len(w1) - 1
    return chi2, dof, stats.chi2.sf(chi2, dof)


def chi2_chunks(a, b, na=1, nb=1, min_frac=0.002):
    """Two-sample test of weighted histograms from independent chunks.

    a, b: arrays (chunks, bins), each row the per-packet histogram (sum over
    the chunk / packets in it) of one chunk of na (resp. nb) packets over
    disjoint photon-id ranges, so rows are independent.  Under the null
    hypothesis both samples draw packets from one distribution, so per bin
    one per-packet variance serves both: it is pooled from the chunks of both
    sides, each squared deviation weighted by its chunk's packet count (a
    chunk mean has variance sigma^2 / n).  The many-packet side then sets the
    estimate, which keeps it from following the few large contributions of
    a small, skewed chunk.  Per bin t = (m_a - m_b) / sqrt(sigma^2 (1/N_a +
    1/N_b)) with K_a + K_b - 2 degrees of freedom is mapped to a standard
    normal quantile through its t distribution, and the squares are summed
    over bins whose pooled mean holds at least `min_frac` of the pooled
    total.  Returns (chi2, dof, p)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    ka, kb = len(a), len(b)
    ma, mb = a.mean(axis=0), b.mean(axis=0)
    s2 = (na * ((a - ma) ** 2).sum(axis=0) + nb * ((b - mb) ** 2).sum(axis=0)) / (ka + kb - 2)
    var = s2 * (1.0 / (ka * na) + 1.0 / (kb * nb))
    tot = ma.sum() + mb.sum()
    sel = ((ma + mb) >= min_frac * tot) & (var > 0)
    t = (ma - mb)[sel] / np.sqrt(var[sel])
    z = stats.norm.isf(stats.t.sf(t, ka + kb - 2))
    chi2 = float(np.sum(z ** 2))
    dof = int(sel.sum())
    return chi2, dof, stats.chi2.sf(chi2, dof)


def rebin(a, factors):
    """Sum blocks of `factors` along each axis (sizes must divide)."""
    a = np.asarray(a)
    shape = []
    for n, f in zip(a.shape, factors):
        assert n % f == 0, (n, f)
        shape += [n // f, f]
    a = a.reshape(shape)
    return a.sum(axis=tuple(range(1, 2 * len(factors), 2)))
