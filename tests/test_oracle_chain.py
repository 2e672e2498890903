"""Pins of the oracle's multi-replica chain: how sweeps, measurements and
exchanges compose (Sec. II, definition of the Monte Carlo step; Eq. (3)).

Each expectation comes from outside the oracle's code path:
  - at beta = 0 every Metropolis proposal is accepted, so after a sweep of one
    Metropolis substep the configuration at beta-position k is the closed form
    theta_i = 2 pi U(a_i(t, k)), with a_i the site's proposal word drawn from
    the independent Python Philox (itself pinned to rocRAND);
  - equal betas make every attempted exchange succeed (exp(0) = 1 > u), so the
    pairs attempted at each step, and therefore the swap counts, are fixed by
    the even/odd schedule alone;
  - at beta = 1e300 a Metropolis move is taken only when it does not raise the
    energy, so that position's energy never increases;
  - with exchange on, each beta-position still samples its own Boltzmann law
    (detailed balance of Eq. (3)), checked against the high-temperature series.
Energies of closed-form states are computed here with numpy rolls from the
definition of Eq. (1).
"""
import numpy as np
import pytest

import oracle.philox_py as P
from stats_util import binned_mean


def energy(theta, L):
    """E = -sum over bonds cos(theta_i - theta_j), each bond once (Eq. (1))."""
    g = theta.reshape(L, L, L)
    return -sum(np.cos(g - np.roll(g, -1, axis=a)).sum() for a in range(3))


def closed_form_beta_zero(L, seed, t, lat, k):
    """Configuration at beta-position k after one beta = 0 Metropolis substep
    (substep index 0) of sweep t."""
    key = P.key_of(seed)
    return np.array([2 * np.pi * P.uniform(P.metro_words(i, L, t, lat, k, 0, key)[0])
                     for i in range(L ** 3)])


def test_each_position_is_measured_before_its_exchange(orc):
    """beta = 0 everywhere, exchange every sweep: the record of sweep s at
    position k is the energy of the closed-form configuration of (t0 + s, k),
    although every attempted pair swaps right after the measurement."""
    L, R, seed, lat, t0, n = 4, 3, 41, 2, 7, 6
    th, obs, _, sacc = orc.run(L, [0.0] * R, seed, n, 1, 0, exchange_every=1, lat=lat, t0=t0)
    cf = {(s, k): closed_form_beta_zero(L, seed, t0 + s, lat, k) for s in range(n) for k in range(R)}
    for s in range(n):
        for k in range(R):
            want = energy(cf[(s, k)], L)
            assert obs[s, k, 0] == pytest.approx(want, abs=1e-9), (s, k)
            assert obs[s, k, 1] == pytest.approx(want / L ** 3, abs=1e-12)
    # the last step (tau = n - 1, odd) swapped pair (1, 2) after the last measurement
    assert np.array_equal(th[0], cf[(n - 1, 0)])
    assert np.array_equal(th[1], cf[(n - 1, 2)])
    assert np.array_equal(th[2], cf[(n - 1, 1)])
    # every attempted pair swapped: pair 0 at even tau, pair 1 at odd tau
    assert sacc.tolist() == [n // 2 + n % 2, n // 2, 0]


@pytest.mark.parametrize("every,n,want", [(1, 5, [3, 2, 0]), (2, 7, [2, 1, 0]), (3, 7, [1, 1, 0]),
                                          (3, 9, [2, 1, 0]), (0, 6, [0, 0, 0])])
def test_exchange_cadence_and_counts(orc, every, n, want):
    """An exchange step follows sweep s when (s + 1) is a multiple of
    exchange_every; with equal betas every attempted pair swaps, so the counts
    follow from the schedule: step tau attempts pair 0 when even, pair 1 when
    odd (R = 3)."""
    L, R = 4, 3
    _, _, _, sacc = orc.run(L, [0.2] * R, 3, n, 1, 1, exchange_every=every)
    assert sacc.tolist() == want


def test_exchange_counts_belong_to_the_attempted_pair(orc):
    """Always-accepted exchanges (Delta >> 0) increment n_acc[k] of the lower
    position k of each attempted pair, and no other entry."""
    L, R = 4, 6
    beta = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6])
    n_acc = np.zeros(R, dtype=np.int64)
    for tau in range(5):
        # E_k = -1e4, E_k+1 = 0 on every pair of this step:
        # (beta_k - beta_k+1)(E_k - E_k+1) = (-0.1)(-1e4) = +1000
        E = np.array([-1e4, 0.0, -1e4, 0.0, -1e4, 0.0]) if tau % 2 == 0 else \
            np.array([0.0, -1e4, 0.0, -1e4, 0.0, 0.0])
        orc.exchange(None, E, L, beta, 11, tau, 0, n_acc)
    # tau = 0, 2, 4 attempt pairs 0, 2, 4; tau = 1, 3 attempt pairs 1, 3
    assert n_acc.tolist() == [3, 2, 3, 2, 3, 0]


def test_each_position_sweeps_at_its_own_beta(orc):
    """Ladder (0, 1e300), no exchange: position 0 is the beta = 0 closed form
    after every sweep, and position 1 (a quench) never raises its energy."""
    L, seed, n = 4, 29, 8
    _, obs, macc, _ = orc.run(L, [0.0, 1e300], seed, n, 1, 0, exchange_every=0)
    for s in range(n):
        assert obs[s, 0, 0] == pytest.approx(energy(closed_form_beta_zero(L, seed, s, 0, 0), L), abs=1e-9)
    E1 = obs[:, 1, 0]
    assert np.all(np.diff(E1) <= 1e-9), E1
    assert macc[0] == n * L ** 3 and 0 < macc[1] < n * L ** 3


def test_tempering_keeps_each_position_at_its_beta(orc):
    """Three positions at beta = 0.05, 0.10, 0.15 with exchange every sweep
    and without: each position's energy and susceptibility match the
    high-temperature series at its own beta, and the two runs agree
    (exchange leaves the product of the Boltzmann laws unchanged)."""
    L, n = 6, 3000
    N = L ** 3
    betas = np.array([0.05, 0.10, 0.15])
    means = {}
    for every in (1, 0):
        _, obs, _, sacc = orc.run(L, betas, 19, n, 1, 1, exchange_every=every)
        if every:
            assert sacc[0] > 100 and sacc[1] > 100  # exchanges do happen
        for k, b in enumerate(betas):
            e_mu, e_err = binned_mean(obs[:, k, 1], discard=0.1)
            c_mu, c_err = binned_mean(N * obs[:, k, 3], discard=0.1)
            want_e = -1.5 * b - 21 / 16 * b ** 3
            want_c = 1 + 3 * b + 7.5 * b ** 2 + 147 / 8 * b ** 3
            assert abs(e_mu - want_e) < 4 * e_err + 10 * b ** 5, (every, k, e_mu, want_e, e_err)
            assert abs(c_mu - want_c) < 4 * c_err + 100 * b ** 4, (every, k, c_mu, want_c, c_err)
            means[(every, k)] = (e_mu, e_err, c_mu, c_err)
    for k in range(3):
        a, b = means[(1, k)], means[(0, k)]
        assert abs(a[0] - b[0]) < 4 * np.hypot(a[1], b[1])
        assert abs(a[2] - b[2]) < 4 * np.hypot(a[3], b[3])
