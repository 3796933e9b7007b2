"""Acceptance statistics for comparing two Monte Carlo dose estimates.

Section 3.1 of the paper: per-voxel t = (D_1 - D_2) / sqrt(sigma_1^2 + sigma_2^2),
two-tailed at significance 0.05, and the passing rate over a dose region; the
mean uncertainty sigma/D_max averaged over voxels with D > 0.5 D_max.  The text
pairs alpha = 0.05 with "90% confidence"; the critical value used here is the
two-tailed alpha = 0.05 quantile of Student's t with N_b - 1 degrees of freedom
(2.262 for N_b = 10), the reading stated in the design notes.
"""
import numpy as np
from scipy import stats as sst


def t_crit(n_batches: int) -> float:
    return float(sst.t.ppf(0.975, n_batches - 1))


def t_values(d1, s1, d2, s2):
    den = np.sqrt(s1 * s1 + s2 * s2)
    with np.errstate(invalid="ignore", divide="ignore"):
        t = np.where(den > 0, (d1 - d2) / den, 0.0)
    return t


def pass_rate(d1, s1, d2, s2, n_batches=10, frac=0.1, mask=None):
    """Fraction of voxels with D > frac * D_max (either estimate) whose |t| < t_crit;
    `mask` restricts both D_max and the region (e.g. to voxels inside the body)."""
    if mask is None:
        mask = np.ones(d1.shape, dtype=bool)
    dmax = max(d1[mask].max(), d2[mask].max())
    region = (np.maximum(d1, d2) > frac * dmax) & mask
    t = t_values(d1, s1, d2, s2)
    ok = np.abs(t[region]) < t_crit(n_batches)
    return float(ok.mean()), int(region.sum())


def unc_over_dmax(dose, sigma, mask=None):
    """Mean of sigma / D_max over voxels with D > 0.5 D_max (section 3.1)."""
    if mask is None:
        mask = np.ones(dose.shape, dtype=bool)
    dmax = dose[mask].max()
    hi = (dose > 0.5 * dmax) & mask
    return float((sigma[hi] / dmax).mean())


def region_sum_test(b1, n1, b2, n2, region):
    """Batch-resolved region sums S_b = sum_{v in region} E_{b,v} / n_b; returns
    (difference of means, combined standard error)."""
    s1 = b1[:, region].sum(axis=1) / n1
    s2 = b2[:, region].sum(axis=1) / n2
    nb1, nb2 = len(s1), len(s2)
    se = np.sqrt(s1.var(ddof=1) / nb1 + s2.var(ddof=1) / nb2)
    return float(s1.mean() - s2.mean()), float(se)
