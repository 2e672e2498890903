"""Statistical pins of the oracle's Markov chain against closed forms.

Each test compares long-run averages of the oracle with a value fixed by the
model itself: exact moments at beta = 0, the single-site von Mises law, the
high-temperature series, the spin-wave limit and the Binder crossing near the
critical point printed in Sec. III.  Seeds are fixed; bounds are 4 sigma (or
4 sigma plus the size of the first neglected series term).
"""
import numpy as np
import pytest
from scipy.special import i0, i1, iv

from stats_util import binned_mean, binned_ratio


def colour_mask(L, c):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return (((x + y + z) & 1) == c).ravel()


@pytest.mark.parametrize("n_or", [0, 3])
def test_beta_zero_exact_moments(orc, n_or):
    """beta = 0: N independent uniform unit vectors.  <e> = 0, Var(e) = 3/(2N),
    N<m^2> = 1, N^2 <m^4> = 2 - 1/N (over-relaxation preserves the law)."""
    L = 8
    N = L ** 3
    _, obs, _, _ = orc.run(L, [0.0], 9, 3000, 1, n_or, exchange_every=0)
    o = obs[:, 0, :]
    e, m2, m4 = o[:, 1], o[:, 3], o[:, 4]
    mu, err = binned_mean(e, discard=0.0)
    assert abs(mu) < 4 * err
    assert abs(e.var() / (3 / (2 * N)) - 1) < 0.1
    mu, err = binned_mean(N * m2, discard=0.0)
    assert abs(mu - 1) < 4 * err
    mu, err = binned_mean(N * N * m4, discard=0.0)
    assert abs(mu - (2 - 1 / N)) < 4 * err


@pytest.mark.parametrize("beta,frozen", [(0.3, 0.0), (1.0, 0.0), (1.0, np.pi / 2)])
def test_single_site_von_mises_law(orc, beta, frozen):
    """Freeze colour 1 at angle a: every colour-0 site sees h = 6 (cos a, sin a),
    so repeated Metropolis half-sweeps on colour 0 sample the von Mises law
    exp(6 beta cos(theta - a)): <cos(theta-a)> = I1/I0, <cos 2(theta-a)> = I2/I0,
    <sin(theta-a)> = 0."""
    L = 6
    N = L ** 3
    th = orc.init(L, 1, 13)[0].copy()
    th[~colour_mask(L, 0)] = frozen
    m0 = colour_mask(L, 0)
    c1, c2, s1 = [], [], []
    for t in range(1500):
        orc.metro_half(th, L, beta, 13, t, 0, 0, 0, 0)
        d = th[m0] - frozen
        c1.append(np.cos(d).mean())
        c2.append(np.cos(2 * d).mean())
        s1.append(np.sin(d).mean())
    k = 6 * beta
    for series, exact in ((c1, i1(k) / i0(k)), (c2, iv(2, k) / i0(k)), (s1, 0.0)):
        mu, err = binned_mean(series, discard=0.1)
        assert abs(mu - exact) < 4 * err + 1e-4, (mu, exact, err)


def test_metropolis_heat_bath_in_random_frozen_field(orc):
    """Colour 1 frozen at random angles: colour-0 site i samples the von Mises
    law of its own field h_i, so <cos(theta_i - phi_i)> = I1(b|h_i|)/I0(b|h_i|),
    with h_i rebuilt here by numpy rolls over the (z, y, x) grid."""
    L, beta = 6, 0.8
    th = orc.init(L, 1, 23)[0].copy()
    g = th.reshape(L, L, L)
    hx = sum(np.cos(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    hy = sum(np.sin(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    m0 = colour_mask(L, 0)
    phi = np.arctan2(hy, hx)[m0]
    h = np.hypot(hx, hy)[m0]
    want = (i1(beta * h) / i0(beta * h)).mean()
    series = []
    for t in range(2000):
        orc.metro_half(th, L, beta, 23, t, 0, 0, 0, 0)
        series.append(np.cos(th[m0] - phi).mean())
    mu, err = binned_mean(series, discard=0.1)
    assert abs(mu - want) < 4 * err + 1e-4


@pytest.mark.slow
@pytest.mark.parametrize("beta", [0.05, 0.1, 0.15])
def test_high_temperature_series(orc, beta):
    """Character expansion: e = -(3/2) b - (21/16) b^3 + O(b^5) and
    N<m^2> = 1 + 3b + (15/2) b^2 + (147/8) b^3 + O(b^4), for L >= 6."""
    L = 8
    N = L ** 3
    _, obs, _, _ = orc.run(L, [beta], 101, 12000, 1, 1, exchange_every=0)
    e = obs[:, 0, 1]
    chi = N * obs[:, 0, 3]
    mu, err = binned_mean(e, discard=0.05)
    want = -1.5 * beta - 21 / 16 * beta ** 3
    assert abs(mu - want) < 4 * err + 10 * beta ** 5, (mu, want, err)
    mu, err = binned_mean(chi, discard=0.05)
    want = 1 + 3 * beta + 7.5 * beta ** 2 + 147 / 8 * beta ** 3
    assert abs(mu - want) < 4 * err + 100 * beta ** 4, (mu, want, err)


@pytest.mark.slow
@pytest.mark.parametrize("beta", [4.0, 8.0])
def test_spin_wave_limit(orc, beta):
    """Low temperature: N - 1 harmonic modes each hold 1/(2 beta), and the
    quartic term of -cos adds 1/(24 beta^2):
    e = -3 + (1 - 1/N)/(2 beta) + 1/(24 beta^2) + O(beta^-3)."""
    L = 6
    N = L ** 3
    _, obs, _, _ = orc.run(L, [beta], 55, 6000, 1, 2, exchange_every=0, ordered=True)
    mu, err = binned_mean(obs[:, 0, 1], discard=0.2)
    want = -3 + (1 - 1 / N) / (2 * beta) + 1 / (24 * beta ** 2)
    assert abs(mu - want) < 4 * err + 0.5 / beta ** 3, (mu, want, err)


@pytest.mark.slow
def test_binder_crossing_brackets_beta_c(orc):
    """Sec. III: U_L curves of different L cross at T_c = 2.2019 (beta_c = 0.4542).
    Below beta_c the larger lattice has the smaller U_L, above it the larger."""
    res = {}
    for beta in (0.42, 0.49):
        for L in (6, 12):
            _, obs, _, _ = orc.run(L, [beta], 7, 3000, 1, 3, exchange_every=0)
            U, err = binned_ratio(obs[:, 0, 4], obs[:, 0, 3],
                                  f=lambda a, b: 1 - a / (3 * b * b))
            res[(beta, L)] = (U, err)
    lo_small, lo_big = res[(0.42, 6)], res[(0.42, 12)]
    hi_small, hi_big = res[(0.49, 6)], res[(0.49, 12)]
    assert lo_small[0] - lo_big[0] > 3 * np.hypot(lo_small[1], lo_big[1])
    assert hi_big[0] - hi_small[0] > 3 * np.hypot(hi_small[1], hi_big[1])


@pytest.mark.parametrize("window", [0.7, 2.5])
def test_windowed_proposal_keeps_the_von_mises_law(orc, window):
    """The restricted-window proposal theta' = theta + w (U - 1/2) is symmetric,
    so the single-site law in a frozen field stays von Mises exp(6 beta cos)."""
    L, beta = 6, 1.0
    th = orc.init(L, 1, 31)[0].copy()
    th[~colour_mask(L, 0)] = 0.0
    m0 = colour_mask(L, 0)
    c1 = []
    for t in range(3000):
        orc.metro_half(th, L, beta, 31, t, 0, 0, 0, 0, window=window)
        c1.append(np.cos(th[m0]).mean())
    k = 6 * beta
    mu, err = binned_mean(c1, discard=0.1)
    assert abs(mu - i1(k) / i0(k)) < 4 * err + 1e-4
