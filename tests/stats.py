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


def batch_doses(batch_edep, rho, vvox, n_per_batch):
    """D_b = E_b / (rho V n_b) per batch and voxel (section 2.2.1)"""
    return batch_edep / (rho * vvox)[None, :] / np.asarray(n_per_batch, dtype=np.float64)[:, None]


def unc_with_jackknife(d_b, mask=None):
    """Mean sigma/D_max (section 3.1) of the batch doses d_b (N_b x voxels)
    and its standard error by the delete-one jackknife over the batches; the
    jackknife sees the correlation between voxels (a batch whose particles
    happen to favour a region moves all its voxels together), which a
    per-voxel error estimate does not."""
    nb = len(d_b)

    def unc(db):
        k = len(db)
        mean = db.mean(axis=0)
        sig = np.sqrt(((db - mean) ** 2).sum(axis=0) / (k * (k - 1)))
        return unc_over_dmax(mean, sig, mask)

    full = unc(d_b)
    # a 9-batch standard error estimates the error of a 9-batch mean: scale
    # the delete-one values to N_b batches before taking their spread
    loo = np.array([unc(np.delete(d_b, b, axis=0)) for b in range(nb)]) * np.sqrt((nb - 1) / nb)
    var = (nb - 1) / nb * ((loo - loo.mean()) ** 2).sum()
    return full, float(np.sqrt(var))
