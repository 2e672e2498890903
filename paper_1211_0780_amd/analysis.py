"""Host-side analysis of measured time series (no GPU work, no Monte Carlo).

The device path records, per sweep and per beta-position, the energy and
magnetisation moments (Eqs. (1), (4)) and the bond sums behind the spin
stiffness (Eq. (6)).  This module turns those series into estimates with
error bars, as the paper does in Sec. II (binning, one-sigma errors) and
Sec. III (Binder cumulant and stiffness crossings, bootstrap resampling):

  binned          mean and error of a correlated series by binning
  jackknife       error of a smooth function of several means
  binder          U_L = 1 - <m^4> / (3 <m^2>^2)            (Eq. (5))
  q2              Q_2 = <m^4> / <m^2>^2 = 3 (1 - U_L)        (Eq. (11))
  stiffness       rho_s = (1/3N) sum_mu [<C_mu> - beta <I_mu^2>]   (Eq. (6))
  crossing        beta where two curves (e.g. U_L or rho_s L for two sizes)
                  cross, by linear interpolation of their difference, with a
                  bootstrap error over the per-beta error bars
  combine_runs    mean of one estimate over independent runs (different
                  seeds) with a standard error from their spread, and how
                  that spread compares with the per-run error bars
  swap_rates      acceptance of each neighbouring pair from exchange counters

The finite-size-scaling fits of Sec. III (data collapse, exponents) need the
paper's production data and are not reproduced here.
"""
import numpy as np


def _trim(x, discard):
    x = np.asarray(x, dtype=np.float64)
    return x[int(len(x) * discard):]


def binned(x, n_bins=20, discard=0.2):
    """(mean, one-sigma error) of a time series: drop the first ``discard``
    fraction, cut the rest into ``n_bins`` consecutive bins, and treat the
    bin means as independent."""
    x = _trim(x, discard)
    nb = len(x) // n_bins
    if nb < 1:
        raise ValueError("series shorter than the number of bins")
    b = x[: nb * n_bins].reshape(n_bins, nb).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(n_bins))


def jackknife(f, *series, n_bins=20, discard=0.2):
    """(value, error) of f(<s1>, <s2>, ...) with leave-one-bin-out jackknife."""
    bins = []
    for s in series:
        s = _trim(s, discard)
        nb = len(s) // n_bins
        if nb < 1:
            raise ValueError("series shorter than the number of bins")
        bins.append(s[: nb * n_bins].reshape(n_bins, nb).mean(axis=1))
    bins = np.stack(bins)
    full = f(*bins.mean(axis=1))
    tot = bins.sum(axis=1)
    jk = np.array([f(*((tot - bins[:, i]) / (n_bins - 1))) for i in range(n_bins)])
    err = np.sqrt((n_bins - 1) / n_bins * ((jk - jk.mean()) ** 2).sum())
    return float(full), float(err)


def binder(m2, m4, **kw):
    """U_L = 1 - <m^4>/(3 <m^2>^2) with the paper's normalisation (Eq. (5))."""
    return jackknife(lambda a, b: 1.0 - b / (3.0 * a * a), m2, m4, **kw)


def q2(m2, m4, **kw):
    """Q_2 = <m^4>/<m^2>^2 (Eq. (11))."""
    return jackknife(lambda a, b: b / (a * a), m2, m4, **kw)


def stiffness(bonds, beta, N, **kw):
    """rho_s of Eq. (6) from a series of bond sums, shape (n_sweeps, 6) with
    columns (C_x, C_y, C_z, I_x, I_y, I_z).  Linear in expectations, so the
    per-sweep estimator (1/3N) sum_mu (C_mu - beta I_mu^2) is averaged."""
    b = np.asarray(bonds, dtype=np.float64)
    per = (b[:, 0:3].sum(axis=1) - beta * (b[:, 3:6] ** 2).sum(axis=1)) / (3.0 * N)
    return binned(per, **kw)


def crossing(betas, ya, ea, yb, eb, n_boot=2000, seed=0):
    """beta at which curve a crosses curve b (a - b changes sign), by linear
    interpolation between the two ladder points that bracket the sign change,
    and its bootstrap spread from Gaussian resampling of every point with its
    error.  Returns (beta_cross, error); (nan, nan) if no sign change."""
    betas = np.asarray(betas, dtype=np.float64)
    ya, ea, yb, eb = (np.asarray(v, dtype=np.float64) for v in (ya, ea, yb, eb))

    def cross(d):
        s = np.sign(d)
        idx = np.flatnonzero(s[:-1] * s[1:] < 0)
        if idx.size == 0:
            return np.nan
        i = idx[np.argmin(np.abs(idx - len(d) / 2))] if idx.size > 1 else idx[0]
        return betas[i] - d[i] * (betas[i + 1] - betas[i]) / (d[i + 1] - d[i])

    b0 = cross(ya - yb)
    if np.isnan(b0):
        return float("nan"), float("nan")
    rng = np.random.default_rng(seed)
    samples = []
    for _ in range(n_boot):
        d = (ya + ea * rng.standard_normal(ya.shape)) - (yb + eb * rng.standard_normal(yb.shape))
        c = cross(d)
        if not np.isnan(c):
            samples.append(c)
    err = float(np.std(samples, ddof=1)) if len(samples) > 1 else float("nan")
    return float(b0), err


def combine_runs(values, errors):
    """Mean over independent runs of an estimate (one per seed), its standard
    error from the spread of the runs, which assumes nothing about the
    per-run error bars (autocorrelation, correlated ladder points), and the
    ratio of that spread to the mean per-run error (about 1 when the per-run
    errors are right).  Returns (mean, standard error, ratio); runs whose
    value is nan (no crossing) are left out, and fewer than two give nan
    for the error and the ratio."""
    v = np.asarray(values, dtype=np.float64)
    e = np.asarray(errors, dtype=np.float64)
    keep = ~np.isnan(v)
    v, e = v[keep], e[keep]
    if v.size == 0:
        return float("nan"), float("nan"), float("nan")
    if v.size < 2:
        return float(v[0]), float("nan"), float("nan")
    sd = float(np.std(v, ddof=1))
    return float(v.mean()), sd / np.sqrt(v.size), sd / float(np.mean(e))


def swap_rates(n_acc, n_exchange_steps, tau0=0):
    """Acceptance rate of each neighbouring pair (k, k+1) of one ladder from
    cumulative swap counts: pair k is attempted at the exchange steps whose
    counter tau has the parity of k."""
    n_acc = np.asarray(n_acc, dtype=np.float64)
    R = len(n_acc)
    taus = np.arange(tau0, tau0 + n_exchange_steps)
    rates = np.full(R - 1, np.nan)
    for k in range(R - 1):
        attempts = int(np.sum((taus & 1) == (k & 1)))
        if attempts:
            rates[k] = n_acc[k] / attempts
    return rates
