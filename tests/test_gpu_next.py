"""GPU tests of the NEXT rows: spin stiffness (Eq. (6)), the finite-size
summary (crossings of U_L and rho_s L, Sec. III) and beta-ladder tuning for
uniform swap acceptance (Sec. II)."""
import numpy as np
import pytest
import torch

from paper_1211_0780_amd import analysis as A
from paper_1211_0780_amd import ladder

pytestmark = pytest.mark.gpu


def make(L, betas, seed, prec="fp32"):
    from paper_1211_0780_amd.sim import Sim
    return Sim(L, betas, seed=seed, prec=prec)


def test_stiffness_inputs_at_beta_zero(gpu):
    """beta = 0: sin(theta_i - theta_j) over distinct bonds are uncorrelated with
    variance 1/2, so <I_mu^2> = N/2 exactly, and <C_mu> = 0."""
    L = 8
    N = L ** 3
    s = make(L, [[0.0]], 21)
    n = 4000
    bonds = torch.zeros((n, 1, 6), dtype=torch.float64, device=gpu)
    s.run(n, 1, 1, exchange_every=0, bonds=bonds)
    b = bonds.cpu().numpy()[:, 0]
    for mu in range(3):
        m, e = A.binned(b[:, 3 + mu] ** 2, discard=0.0)
        assert abs(m - N / 2) < 4 * e
        m, e = A.binned(b[:, mu], discard=0.0)
        assert abs(m) < 4 * e


def test_stiffness_ordered_limit(gpu):
    """Ordered state: C_mu = N, I_mu = 0, so rho_s = 1.  At large beta the
    harmonic bond variance 1/(3 beta) gives <cos> ~ 1 - 1/(6 beta), and the
    linear part of I_mu telescopes to zero under periodic boundaries, so
    rho_s ~ 1 - 1/(6 beta) up to higher orders (checked loosely)."""
    L, beta = 8, 6.0
    s = make(L, [[beta]], 2)
    s.set_angles(np.zeros(L ** 3))
    b = s.bond_sums()[0]
    assert np.allclose(b[:3], L ** 3) and np.allclose(b[3:], 0.0, atol=1e-6)
    n = 3000
    bonds = torch.zeros((n, 1, 6), dtype=torch.float64, device=gpu)
    s.run(n, 1, 2, exchange_every=0, bonds=bonds)
    rho, err = A.stiffness(bonds.cpu().numpy()[:, 0], beta, L ** 3)
    assert 0.8 < rho < 1.0


def test_fss_summary_crossings(gpu):
    """rho_s L and U_L for L = 8 and 16 over a ladder straddling beta_c cross
    inside it (Sec. III: both cross at T_c = 2.2019, beta_c = 0.4542)."""
    from paper_1211_0780_amd.fss import run_batch
    betas = np.linspace(0.42, 0.49, 8)
    res = run_batch([8, 16], betas, seed=3, n_sweeps=4000, n_or=4)
    print("[fss-lite] crossings", res["crossings"], "rate", res["site_updates_per_s"])
    for c in res["crossings"]:
        assert 0.42 < c["beta_cross"] < 0.49, c
    lo = res["per_L"]["8"]["rows"][0]["U"][0] - res["per_L"]["16"]["rows"][0]["U"][0]
    hi = res["per_L"]["8"]["rows"][-1]["U"][0] - res["per_L"]["16"]["rows"][-1]["U"][0]
    assert lo > 0 > hi


def test_ladder_tuning_flattens_swap_acceptance(gpu):
    """Measure pair acceptances on a linear ladder that straddles the
    transition, respace it, measure again: the spread shrinks."""
    L, R, n = 10, 8, 3000
    betas = np.linspace(0.30, 0.60, R)
    spreads = []
    for it in range(3):
        s = make(L, [betas], 7 + it)
        s.run(n, 1, 2, exchange_every=1)
        rates = A.swap_rates(s.swap_accepts(), n)
        spreads.append(np.ptp(rates))
        print(f"[ladder] iteration {it}: betas {np.round(betas, 4)} rates {np.round(rates, 3)}")
        s.close()
        betas = ladder.respace(betas, rates)
    assert spreads[-1] < 0.6 * spreads[0]
