"""Deterministic pins of the oracle's update and measurement steps.

Every expectation here comes from the mathematics of the model, computed
independently of the oracle's code path: neighbour fields are rebuilt with
numpy rolls over the (z, y, x) grid, closed forms come from special states.
"""
import numpy as np
import pytest

import oracle.philox_py as P


def grid(theta, L):
    return theta.reshape(L, L, L)  # [z, y, x]


def colour_mask(L, c):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return ((x + y + z) & 1) == c


def field(theta, L):
    """Sum of the six neighbouring unit vectors, by numpy rolls (periodic)."""
    g = grid(theta, L)
    hx = np.zeros_like(g)
    hy = np.zeros_like(g)
    for ax in range(3):
        for sh in (1, -1):
            r = np.roll(g, sh, axis=ax)
            hx += np.cos(r)
            hy += np.sin(r)
    return hx, hy


def circ(a, b):
    d = np.abs(np.asarray(a) - np.asarray(b)) % (2 * np.pi)
    return np.minimum(d, 2 * np.pi - d)


def test_beta_zero_metropolis_accepts_every_proposal(orc):
    """At beta = 0, exp(-beta dE) = 1 > u, so every site takes theta' = 2 pi U(a), a its proposal word."""
    L, seed, t, lat, k, s = 6, 77, 5, 1, 3, 2
    th = orc.init(L, 1, seed, lat)[0].copy()
    key = P.key_of(seed)
    for c in (0, 1):
        acc = orc.metro_half(th, L, 0.0, seed, t, lat, k, s, c)
        assert acc == L ** 3 // 2
    for i in range(L ** 3):
        a, _ = P.metro_words(i, L, t, lat, k, s, key)
        assert th[i] == 2 * np.pi * P.uniform(a)


def test_metropolis_only_touches_its_colour(orc):
    L = 6
    th0 = orc.init(L, 1, 5)[0].copy()
    for c in (0, 1):
        th = th0.copy()
        orc.metro_half(th, L, 0.45, 5, 0, 0, 0, 0, c)
        other = ~colour_mask(L, c).ravel()
        assert np.array_equal(th[other], th0[other])
        assert np.any(th[~other] != th0[~other])


def test_metropolis_decisions_follow_local_energy(orc):
    """Each accepted/rejected move agrees with u < exp(-beta dE), dE from the
    vector form (S - S').h with h from numpy rolls."""
    L, seed, t, lat, k, s, beta = 6, 11, 3, 0, 2, 0, 0.7
    th0 = orc.init(L, 1, seed)[0].copy()
    for c in (0, 1):
        th = th0.copy()
        orc.metro_half(th, L, beta, seed, t, lat, k, s, c)
        hx, hy = field(th0, L)
        hx, hy = hx.ravel(), hy.ravel()
        key = P.key_of(seed)
        n_checked = 0
        for i in np.flatnonzero(colour_mask(L, c).ravel()):
            a, b = P.metro_words(int(i), L, t, lat, k, s, key)
            prop = 2 * np.pi * P.uniform(a)
            u = P.uniform(b)
            dE = (np.cos(th0[i]) - np.cos(prop)) * hx[i] + (np.sin(th0[i]) - np.sin(prop)) * hy[i]
            p = np.exp(-beta * dE)
            if abs(u - p) < 1e-12:
                continue
            expect = prop if u < p else th0[i]
            assert th[i] == expect, i
            n_checked += 1
        assert n_checked > 0.9 * L ** 3 / 2
        th0 = th  # colour 1 sees the updated colour 0


def test_overrelaxation_is_reflection_about_field(orc):
    """Eq. (2): S' is S reflected about the line of H, so relative to the field
    direction phi the angle flips sign: theta' - phi = -(theta - phi)."""
    L = 6
    th0 = orc.init(L, 1, 21)[0].copy()
    for c in (0, 1):
        th = th0.copy()
        orc.or_half(th, L, c)
        hx, hy = field(th0, L)
        phi = np.arctan2(hy, hx).ravel()
        m = colour_mask(L, c).ravel()
        assert np.max(circ(th[m] - phi[m], -(th0[m] - phi[m]))) < 1e-12
        assert np.array_equal(th[~m], th0[~m])
        assert th.min() >= 0 and th.max() < 2 * np.pi
        th0 = th


def test_overrelaxation_is_an_involution(orc):
    L = 8
    th0 = orc.init(L, 1, 4)[0].copy()
    for c in (0, 1):
        th = th0.copy()
        orc.or_half(th, L, c)
        orc.or_half(th, L, c)
        assert np.max(circ(th, th0)) < 1e-12


def test_overrelaxation_conserves_energy(orc):
    """The over-relaxation move is microcanonical (Sec. II)."""
    L = 8
    th = orc.init(L, 1, 8)[0].copy()
    # move away from the random start so the state has structure
    orc.sweep(th, L, [0.6], 8, 0, 0, 3, 0)
    E0 = orc.measure(th, L)[0]
    for _ in range(20):
        orc.or_half(th, L, 0)
        orc.or_half(th, L, 1)
    assert abs(orc.measure(th, L)[0] - E0) < 1e-9 * L ** 3


def test_ordered_state(orc):
    L = 6
    N = L ** 3
    for a in (0.0, 1.234, 5.9):
        th = np.full(N, a)
        E, e, m, m2, m4 = orc.measure(th, L)
        assert E == pytest.approx(-3 * N, abs=1e-9)
        assert m == pytest.approx(1.0, abs=1e-12)
        assert m2 == pytest.approx(1.0, abs=1e-12) and m4 == pytest.approx(1.0, abs=1e-12)
        th2 = th.copy()
        orc.or_half(th2, L, 0)
        orc.or_half(th2, L, 1)
        assert np.max(circ(th2, th)) < 1e-12
        C = orc.bond_sums(th, L)
        assert np.allclose(C[:3], N) and np.allclose(C[3:], 0, atol=1e-9)


def test_global_rotation_invariance(orc):
    L = 6
    th = orc.init(L, 1, 31)[0]
    a = orc.measure(th, L)
    b = orc.measure((th + 2.2) % (2 * np.pi), L)
    assert a[0] == pytest.approx(b[0], abs=1e-10)
    assert a[2] == pytest.approx(b[2], abs=1e-13)


@pytest.mark.parametrize("q", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (1, 2, 3)])
def test_spin_wave_closed_forms(orc, q):
    """theta = 2 pi (q . r)/L: E = -N sum_mu cos(2 pi q_mu / L), M = 0 unless q = 0,
    C_mu = N cos(2 pi q_mu / L), I_mu = -N sin(2 pi q_mu / L)."""
    L = 8
    N = L ** 3
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    th = (2 * np.pi * (q[0] * x + q[1] * y + q[2] * z) / L) % (2 * np.pi)
    th = th.ravel().astype(np.float64)
    a = 2 * np.pi * np.array(q) / L
    E, e, m, m2, m4 = orc.measure(th, L)
    assert E == pytest.approx(-N * np.cos(a).sum(), abs=1e-9)
    assert m == pytest.approx(0.0, abs=1e-12)
    C = orc.bond_sums(th, L)
    assert np.allclose(C[:3], N * np.cos(a), atol=1e-9)
    assert np.allclose(C[3:], -N * np.sin(a), atol=1e-9)


def test_two_sublattice_antiparallel_state(orc):
    """Colour 0 at alpha, colour 1 at alpha + pi: every bond costs +1, m = 0."""
    L = 6
    N = L ** 3
    th = np.where(colour_mask(L, 0).ravel(), 0.7, 0.7 + np.pi)
    E, e, m, m2, m4 = orc.measure(th, L)
    assert E == pytest.approx(3 * N, abs=1e-9)
    assert m == pytest.approx(0.0, abs=1e-12)


def test_exchange_rules(orc):
    """Eq. (3): W = min[1, exp((beta_k - beta_k+1)(E_k - E_k+1))], pairs alternate."""
    L, N, seed = 4, 64, 3
    R = 6
    beta = np.array([0.1, 0.1, 0.2, 0.3, 0.4, 0.5])
    # equal betas: always swap pair (0, 1) at even tau
    theta = np.arange(R * N, dtype=np.float64).reshape(R, N).copy()
    E = np.array([-10.0, -20.0, 0.0, 0.0, 0.0, 0.0])
    n_acc = np.zeros(R, dtype=np.int64)
    orc.exchange(theta, E, L, beta, seed, 0, 0, n_acc)
    assert E[0] == -20.0 and E[1] == -10.0
    assert theta[0, 0] == N and theta[1, 0] == 0
    # the odd step pairs (1,2),(3,4) only
    E = np.array([0.0, -100.0, 100.0, -100.0, 100.0, 0.0])
    # (beta1-beta2)(E1-E2) = (-0.1)(-200) = +20 -> always; same for (3,4)
    E0 = E.copy()
    orc.exchange(None, E, L, beta, seed, 1, 0, None)
    assert E[1] == E0[2] and E[2] == E0[1] and E[3] == E0[4] and E[4] == E0[3]
    assert E[0] == E0[0] and E[5] == E0[5]
    # strongly unfavourable pairs never swap; the equal-beta pair (0, 1) always does
    for tau in range(0, 40, 2):
        Ec = np.array([1000.0, -1000.0, 1000.0, -1000.0, 1000.0, -1000.0])
        Ecopy = Ec.copy()
        orc.exchange(None, Ec, L, beta, seed, tau, 0, None)
        # pairs (2,3), (4,5): (-0.1)(2000) = -200
        assert np.array_equal(Ec[2:], Ecopy[2:])
        assert Ec[0] == Ecopy[1]


def test_exchange_acceptance_rate(orc):
    """Intermediate Delta: acceptance fraction equals exp(Delta) within binomial error."""
    L = 4
    beta = np.array([0.40, 0.45])
    delta = -0.7
    dE = delta / (beta[0] - beta[1])
    n, acc = 4000, 0
    for tau in range(0, 2 * n, 2):
        E = np.array([dE, 0.0])
        acc += orc.exchange(None, E, L, beta, 17, tau, 0, None)
    p = np.exp(delta)
    assert abs(acc / n - p) < 4 * np.sqrt(p * (1 - p) / n)


def test_windowed_metropolis_proposal_and_decisions(orc):
    """Window w: proposal wrap(theta + w (U(a) - 1/2)), decided by u < exp(-beta dE)."""
    L, seed, t, lat, k, s, beta, w = 6, 12, 4, 0, 1, 0, 0.6, 1.3
    th0 = orc.init(L, 1, seed)[0].copy()
    th = th0.copy()
    orc.metro_half(th, L, beta, seed, t, lat, k, s, 0, window=w)
    hx, hy = field(th0, L)
    hx, hy = hx.ravel(), hy.ravel()
    key = P.key_of(seed)
    moved = 0
    for i in np.flatnonzero(colour_mask(L, 0).ravel()):
        a, b = P.metro_words(int(i), L, t, lat, k, s, key)
        prop = (th0[i] + w * (P.uniform(a) - 0.5)) % (2 * np.pi)
        u = P.uniform(b)
        dE = (np.cos(th0[i]) - np.cos(prop)) * hx[i] + (np.sin(th0[i]) - np.sin(prop)) * hy[i]
        p = np.exp(-beta * dE)
        if abs(u - p) < 1e-12:
            continue
        if u < p:
            assert circ(th[i], prop) < 1e-13
            moved += 1
        else:
            assert th[i] == th0[i]
    assert moved > 0


@pytest.mark.parametrize("window", [0.0, 1.3])
def test_metropolis_margins(orc, window):
    """orc.metro_margin gives U(b) - exp(-beta dE) for every site of the
    colour, with the proposal word, the acceptance word and dE rebuilt here
    from the Python Philox and numpy-rolled fields; NaN on the other colour."""
    L, seed, t, lat, k, s, beta = 6, 21, 2, 1, 3, 1, 0.55
    th0 = orc.init(L, 1, seed, lat)[0].copy()
    key = P.key_of(seed)
    hx, hy = field(th0, L)
    hx, hy = hx.ravel(), hy.ravel()
    for c in (0, 1):
        m = orc.metro_margin(th0, L, beta, seed, t, lat, k, s, c, window=window)
        mask = colour_mask(L, c).ravel()
        assert np.all(np.isnan(m[~mask])) and not np.any(np.isnan(m[mask]))
        for i in np.flatnonzero(mask):
            a, b = P.metro_words(int(i), L, t, lat, k, s, key)
            prop = (th0[i] + window * (P.uniform(a) - 0.5)) % (2 * np.pi) if window else 2 * np.pi * P.uniform(a)
            dE = (np.cos(th0[i]) - np.cos(prop)) * hx[i] + (np.sin(th0[i]) - np.sin(prop)) * hy[i]
            assert m[i] == pytest.approx(P.uniform(b) - np.exp(-beta * dE), abs=1e-12), i
        # and the half-sweep takes exactly the moves with a negative margin
        th = th0.copy()
        orc.metro_half(th, L, beta, seed, t, lat, k, s, c, window=window)
        assert np.array_equal(th[mask] != th0[mask], m[mask] < 0)
