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
