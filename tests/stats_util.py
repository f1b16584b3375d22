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
