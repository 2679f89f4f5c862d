"""Two-sample statistics for Monte Carlo tallies (test helpers)."""
from __future__ import annotations

import numpy as np


def chi2_two_sample(n1, n2, min_count=20):
    """Two-sample chi^2 of histograms with totals N1, N2 over bins where both
    samples expect >= min_count counts under the pooled proportion (so the
    normal approximation behind chi^2 and z holds in each).  Returns (chi2, dof,
    max|z|)."""
    n1 = np.asarray(n1, dtype=np.float64)
    n2 = np.asarray(n2, dtype=np.float64)
    N1, N2 = n1.sum(), n2.sum()
    m = (n1 + n2) / (N1 + N2) * min(N1, N2) >= min_count
    a, b = n1[m], n2[m]
    k1, k2 = np.sqrt(N2 / N1), np.sqrt(N1 / N2)
    chi2 = float(np.sum((k1 * a - k2 * b) ** 2 / (a + b)))
    p1, p2 = a / N1, b / N2
    z = (p1 - p2) / np.sqrt(a / N1 ** 2 + b / N2 ** 2)
    return chi2, int(m.sum()) - 1, float(np.max(np.abs(z))) if z.size else 0.0


def l1_shape(n1, n2):
    """L1 distance of the two normalised histograms (sum |p1 - p2|)."""
    p1 = np.asarray(n1, dtype=np.float64)
    p2 = np.asarray(n2, dtype=np.float64)
    return float(np.abs(p1 / p1.sum() - p2 / p2.sum()).sum())


def l1_floor(p, N1, N2, trials=200, seed=123):
    """Expected L1 between two multinomial samples of sizes N1, N2 from p."""
    rng = np.random.default_rng(seed)
    p = np.asarray(p, dtype=np.float64)
    p = p / p.sum()
    vals = [l1_shape(rng.multinomial(N1, p), rng.multinomial(N2, p)) for _ in range(trials)]
    return float(np.mean(vals)), float(np.std(vals))


def ks_two_sample(x, y):
    from scipy.stats import ks_2samp
    return ks_2samp(x, y)
