"""Host-side analysis (binning, Binder, Q2, stiffness, crossings, swap rates)
and ladder tuning, on synthetic series with known answers."""
import numpy as np
import pytest

from paper_1211_0780_amd import analysis as A
from paper_1211_0780_amd import ladder


def test_binned_mean_and_error_of_ar1_series():
    rng = np.random.default_rng(0)
    n, phi = 200_000, 0.9
    x = np.empty(n)
    x[0] = 0.0
    eps = rng.standard_normal(n)
    for i in range(1, n):
        x[i] = phi * x[i - 1] + eps[i]
    mu, err = A.binned(x + 3.0, n_bins=40, discard=0.0)
    # exact error of the mean of an AR(1) series: sqrt(var * (1+phi)/(1-phi) / n)
    exact = np.sqrt(1 / (1 - phi ** 2) * (1 + phi) / (1 - phi) / n)
    assert abs(mu - 3.0) < 4 * exact
    assert 0.6 * exact < err < 1.5 * exact


def test_binder_and_q2_of_known_moments():
    rng = np.random.default_rng(1)
    # m distributed so that <m^2> = 1, <m^4> = 2 (2D Gaussian magnetisation)
    v = rng.standard_normal((100_000, 2)) / np.sqrt(2)
    m2 = (v ** 2).sum(axis=1)
    m4 = m2 ** 2
    U, eU = A.binder(m2, m4, discard=0.0)
    Q, eQ = A.q2(m2, m4, discard=0.0)
    assert abs(U - (1 - 2 / 3)) < 4 * eU
    assert abs(Q - 2.0) < 4 * eQ
    assert abs(Q - 3 * (1 - U)) < 1e-12


def test_stiffness_estimator():
    N, beta = 1000, 0.5
    b = np.zeros((100, 6))
    b[:, 0:3] = 600.0          # <C_mu> = 600
    b[:, 3:6] = 10.0           # I_mu^2 = 100
    rho, err = A.stiffness(b, beta, N, discard=0.0)
    assert rho == pytest.approx((3 * 600 - beta * 3 * 100) / (3 * N))
    assert err < 1e-12


def test_crossing_of_two_lines():
    betas = np.linspace(0.44, 0.47, 7)
    ya = 0.5 + 2.0 * (betas - 0.4542)
    yb = 0.5 + 9.0 * (betas - 0.4542)
    e = np.full_like(betas, 1e-3)
    bc, err = A.crossing(betas, ya, e, yb, e)
    assert bc == pytest.approx(0.4542, abs=1e-9)
    assert 0 < err < 1e-3
    assert np.isnan(A.crossing(betas, ya, e, ya + 1, e)[0])


def test_precision_ensemble_binder_jackknife():
    """The ensemble study's U_L error: with m^2 the same in every ladder U_L
    is linear in the mean of m^4, and the leave-one-ladder-out jackknife of a
    linear function of a mean is exactly its standard error; identical
    ladders give no error and the closed form of Eq. (5)."""
    from paper_1211_0780_amd import precision as P
    rng = np.random.default_rng(3)
    K, R = 9, 4
    m = np.zeros((K, R, 5))
    m[:, :, 3] = 0.02
    m[:, :, 4] = 6e-4 + 1e-5 * rng.standard_normal((K, R))
    u, err = P._binder_jk(m)
    assert np.allclose(u, 1.0 - m[:, :, 4].mean(0) / (3 * 0.02 ** 2), rtol=0, atol=1e-15)
    se = m[:, :, 4].std(0, ddof=1) / np.sqrt(K) / (3 * 0.02 ** 2)
    assert np.allclose(err, se, rtol=1e-10)
    same = np.repeat(m[:1], K, axis=0)
    u1, e1 = P._binder_jk(same)
    assert np.allclose(u1, 1.0 - same[0, :, 4] / (3 * same[0, :, 3] ** 2)) and np.all(e1 < 1e-15)
    with pytest.raises(ValueError):
        P.compare_ladders(8, [0.45, 0.46], n32=1, n64=4)


def test_combine_runs_of_known_spread():
    # 400 runs of an estimate 0.4542 + N(0, 2e-4) whose per-run error bars
    # claim 1e-4: the spread is twice the claim
    rng = np.random.default_rng(11)
    v = 0.4542 + 2e-4 * rng.standard_normal(400)
    m, se, ratio = A.combine_runs(v, np.full(400, 1e-4))
    assert m == pytest.approx(0.4542, abs=4 * 2e-4 / 20)
    assert se == pytest.approx(2e-4 / 20, rel=0.1)
    assert ratio == pytest.approx(2.0, rel=0.1)
    # exact small case and the nan handling
    m, se, ratio = A.combine_runs([1.0, 3.0, np.nan], [1.0, 1.0, 5.0])
    assert (m, se, ratio) == pytest.approx((2.0, 1.0, np.sqrt(2.0)))
    m, se, ratio = A.combine_runs([1.0], [0.5])
    assert m == 1.0 and np.isnan(se) and np.isnan(ratio)


def test_swap_rates_parity_bookkeeping():
    # pairs 0, 2 attempted on even tau, 1 on odd tau; 10 exchange steps
    rates = A.swap_rates([5, 2, 5, 0], 10)
    assert np.allclose(rates, [1.0, 0.4, 1.0])


def test_ladder_respacing_equalises_model_acceptance():
    sigma = lambda b: 60.0 * (1.0 + 400.0 * (b - 0.45) ** 2)
    betas = np.linspace(0.40, 0.50, 12)
    spread0 = np.ptp(ladder.predicted_acceptance(betas, sigma))
    for _ in range(6):
        betas = ladder.respace(betas, ladder.predicted_acceptance(betas, sigma))
    acc = ladder.predicted_acceptance(betas, sigma)
    assert betas[0] == 0.40 and betas[-1] == 0.50 and np.all(np.diff(betas) > 0)
    assert np.ptp(acc) < 0.01 < 0.1 < spread0


def test_ladder_rejects_bad_input():
    with pytest.raises(ValueError):
        ladder.respace([0.1, 0.1, 0.2], [0.5, 0.5])
    with pytest.raises(ValueError):
        ladder.respace([0.1, 0.2], [0.5, 0.5])


def test_fss_combine_crossings_over_seeds():
    from paper_1211_0780_amd.fss import combine_crossings
    runs = [{"crossings": [{"pair": [8, 16], "quantity": "U", "beta_cross": b, "err": 1e-4},
                           {"pair": [8, 16], "quantity": "rhoL", "beta_cross": float("nan"), "err": float("nan")}]}
            for b in (0.4540, 0.4542, 0.4544)]
    c = combine_crossings(runs)
    assert [x["quantity"] for x in c] == ["U", "rhoL"]
    assert c[0]["beta_cross"] == pytest.approx(0.4542)
    assert c[0]["err"] == pytest.approx(2e-4 / np.sqrt(3))
    assert c[0]["spread_over_quoted"] == pytest.approx(2.0)
    assert c[0]["n_runs"] == 3 and len(c[0]["per_run"]) == 3
    assert np.isnan(c[1]["beta_cross"])
