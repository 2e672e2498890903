"""Small statistics helpers for the statistical tests (binning error bars)."""
import numpy as np


def binned_mean(x, n_bins=20, discard=0.2):
    """Mean and one-sigma error of a correlated time series by binning.

    The first ``discard`` fraction is dropped as equilibration; the rest is cut
    into ``n_bins`` consecutive bins whose means are treated as independent.
    """
    x = np.asarray(x, dtype=np.float64)
    x = x[int(len(x) * discard):]
    nb = len(x) // n_bins
    if nb < 1:
        raise ValueError("series too short for binning")
    b = x[: nb * n_bins].reshape(n_bins, nb).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(n_bins)


def binned_ratio(num, den, n_bins=20, discard=0.2, f=lambda a, b: a / b):
    """f(<num>, <den>) with a jackknife error over bins."""
    num = np.asarray(num, dtype=np.float64)
    den = np.asarray(den, dtype=np.float64)
    s = int(len(num) * discard)
    num, den = num[s:], den[s:]
    nb = len(num) // n_bins
    bn = num[: nb * n_bins].reshape(n_bins, nb).mean(axis=1)
    bd = den[: nb * n_bins].reshape(n_bins, nb).mean(axis=1)
    full = f(bn.mean(), bd.mean())
    jk = np.array([f(np.delete(bn, i).mean(), np.delete(bd, i).mean()) for i in range(n_bins)])
    err = np.sqrt((n_bins - 1) / n_bins * ((jk - jk.mean()) ** 2).sum())
    return full, err


def bonferroni_z(n, alpha=0.05):
    """Two-sided gate for a family of n comparisons at family-wise error
    alpha: Phi^-1(1 - alpha / (2 n)).  n = 5: 2.58; 20: 3.02; 80: 3.42; 160: 3.60."""
    from scipy.special import ndtri
    return float(ndtri(1.0 - alpha / (2.0 * n)))


def chain_bins(x, n_bins=20, discard=0.2):
    """Bin means of one chain's series after dropping the first `discard`."""
    x = np.asarray(x, dtype=np.float64)
    x = x[int(len(x) * discard):]
    nb = len(x) // n_bins
    if nb < 1:
        raise ValueError("series too short for binning")
    return x[: nb * n_bins].reshape(n_bins, nb).mean(axis=1)


def bins_mean(b):
    b = np.asarray(b, dtype=np.float64)
    return b.mean(), b.std(ddof=1) / np.sqrt(b.size)


def bins_ratio(bn, bd, f):
    """f(<num>, <den>) with a jackknife error over paired bins."""
    bn, bd = np.asarray(bn, dtype=np.float64), np.asarray(bd, dtype=np.float64)
    n = bn.size
    full = f(bn.mean(), bd.mean())
    sn, sd = bn.sum(), bd.sum()
    jk = f((sn - bn) / (n - 1), (sd - bd) / (n - 1))
    err = np.sqrt((n - 1) / n * ((jk - jk.mean()) ** 2).sum())
    return float(full), float(err)


def binder(m4, m2):
    """U_L = 1 - <m^4> / (3 <m^2>^2) (Eq. (5), the paper's factor 3)."""
    return 1.0 - m4 / (3.0 * m2 * m2)


def z_family(pairs):
    """z-scores of (mean_a, err_a, mean_b, err_b) tuples, with the fraction
    within 2 sigma (expected about 0.95 for independent comparisons)."""
    z = np.array([(a - b) / np.hypot(ea, eb) for a, ea, b, eb in pairs])
    return z, float(np.mean(np.abs(z) <= 2.0))
