"""Temperature-ladder tuning for parallel tempering (host side).

Sec. II chooses the temperature set so that the swap acceptance between
neighbouring temperatures does not depend on the temperature.  This module
does that by feedback: from the measured acceptance A_k of each neighbouring
pair of a ladder, estimate the local energy spread, then place a new ladder
(same end points, same length) at equal steps of the accumulated spread.

Model: for a pair at inverse temperatures beta and beta + d whose energy
distributions are close to Gaussian with width sigma, the swap acceptance of
Eq. (3) is about erfc(d * sigma / 2).  Inverting it on each gap gives
sigma_k = 2 erfcinv(A_k) / d_k, a piecewise-constant density on [beta_0,
beta_max]; new points are equally spaced in S(beta) = integral of sigma, so
every new gap has the same d * sigma and, under the model, the same
acceptance.  A few rounds of measure-and-respace converge.
"""
import numpy as np
from scipy.special import erfcinv


def respace(betas, acceptance, clip=(1e-3, 1 - 1e-3)):
    """New ladder with the same end points and length whose predicted pair
    acceptances are equal.  ``acceptance`` has len(betas) - 1 entries."""
    b = np.asarray(betas, dtype=np.float64)
    A = np.clip(np.asarray(acceptance, dtype=np.float64), *clip)
    if b.ndim != 1 or len(A) != len(b) - 1:
        raise ValueError("need R betas and R-1 acceptances")
    d = np.diff(b)
    if np.any(d <= 0):
        raise ValueError("betas must be strictly ascending")
    sigma = 2.0 * erfcinv(A) / d
    S = np.concatenate([[0.0], np.cumsum(sigma * d)])
    targets = np.linspace(0.0, S[-1], len(b))
    new = np.interp(targets, S, b)
    new[0], new[-1] = b[0], b[-1]
    return new


def predicted_acceptance(betas, sigma_of_beta):
    """Acceptances erfc(d sigma(mid)/2) of a ladder under a given width
    function (used to check the construction)."""
    from scipy.special import erfc
    b = np.asarray(betas, dtype=np.float64)
    mid = 0.5 * (b[1:] + b[:-1])
    return erfc(np.diff(b) * sigma_of_beta(mid) / 2.0)
