"""Long-run statistical parity (same equilibrium law) on the GPU.

GPU chains against the oracle's chain (the L = 8 single lattice, and a
small parallel-tempering ladder), float32 against float64 kernels on the
same ladders, exchange on against off, and the Binder crossing of the
batched finite-size-scaling set.  The two chains of a comparison always run
from different seeds, so they are independent samples of the same law.
Averages use binning (20 bins after discarding 20 % as equilibration); the
z-score of a comparison is (a - b) / sqrt(sa^2 + sb^2).  Each test is one
family of n comparisons (positions x observables) gated at its Bonferroni
bound Phi^-1(1 - 0.025 / n) (family-wise error 5 %: 2.58 for n = 5, 3.02 for
20, 3.60 for 160); the largest |z| and the fraction within 2 sigma (about
0.95 expected for independent comparisons) are printed for the record.
"""
import numpy as np
import pytest
import torch

import oracle
from stats_util import binned_mean, binned_ratio, bonferroni_z, z_family

pytestmark = pytest.mark.gpu


def make(L, betas, seed, prec="fp32", start="random"):
    from paper_1211_0780_amd.sim import Sim
    return Sim(L, betas, seed=seed, prec=prec, start=start)


def gpu_series(sim, n, n_metro, n_or, exchange_every):
    obs = torch.zeros((n, sim.R_total, 5), dtype=torch.float64, device="cuda")
    sim.run(n, n_metro, n_or, exchange_every=exchange_every, obs=obs)
    torch.cuda.synchronize()
    return obs.cpu().numpy()


def summary(o):
    """Per position: (mean, err) of e, |m|, m^2, m^4 and U_L."""
    out = []
    for p in range(o.shape[1]):
        row = [binned_mean(o[:, p, c]) for c in (1, 2, 3, 4)]
        row.append(binned_ratio(o[:, p, 4], o[:, p, 3], f=lambda a, b: 1 - a / (3 * b * b)))
        out.append(row)
    return out


def compare(a, b, label):
    """Gate the family of comparisons a vs b at its Bonferroni bound."""
    names = ("e", "|m|", "m2", "m4", "U_L")
    pairs, labels = [], []
    for p, (ra, rb) in enumerate(zip(a, b)):
        for name, (ma, ea), (mb, eb) in zip(names, ra, rb):
            pairs.append((ma, ea, mb, eb))
            labels.append(f"pos {p} {name}")
    z, frac2 = z_family(pairs)
    gate = bonferroni_z(len(pairs))
    worst = int(np.argmax(np.abs(z)))
    print(f"[{label}] {len(pairs)} comparisons: max |z| = {abs(z[worst]):.2f} ({labels[worst]}), "
          f"within 2 sigma {frac2:.3f}, gate {gate:.2f}")
    bad = [f"{labels[i]}: z = {z[i]:.2f}" for i in np.flatnonzero(np.abs(z) > gate)]
    assert not bad, f"{label}: {bad}"
    return float(np.abs(z).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_lattice_long_run_matches_oracle(gpu, prec):
    """L = 8, beta = 0.4542, 1 Metropolis + 1 over-relaxation, 10^4 sweeps.
    The oracle's chain runs from another seed: with the same seed the two
    chains would follow one trajectory and the comparison would be empty."""
    L, beta, seed, n = 8, 0.4542, 1, 10000
    s = make(L, [[beta]], seed, prec)
    og = gpu_series(s, n, 1, 1, 0)
    _, oo, _, _ = oracle.run(L, [beta], seed + 1000, n, 1, 1, exchange_every=0)
    compare(summary(og), summary(oo), f"L=8 {prec} vs oracle")


def test_tempering_ladder_long_run_matches_oracle(gpu):
    """L = 8, four replicas over [0.40, 0.50], exchange every sweep, FP32."""
    L, seed, n = 8, 2, 10000
    betas = list(np.linspace(0.40, 0.50, 4))
    s = make(L, [betas], seed)
    og = gpu_series(s, n, 1, 2, 1)
    _, oo, _, sacc = oracle.run(L, betas, seed + 1000, n, 1, 2, exchange_every=1)
    compare(summary(og), summary(oo), "L=8 PT fp32 vs oracle")


def test_exchange_does_not_change_equilibrium(gpu):
    L, n = 12, 8000
    betas = list(np.linspace(0.42, 0.48, 6))
    a = gpu_series(make(L, [betas], 11), n, 1, 3, 1)
    b = gpu_series(make(L, [betas], 12), n, 1, 3, 0)
    compare(summary(a), summary(b), "PT on vs off")


def test_fp32_matches_fp64_on_a_ladder(gpu):
    """The L = 64 ladder: 32 replicas over [0.4530, 0.4554], 1 + 8,
    float32 (with float64 near-threshold re-decision) against the all-float64
    kernels, both with exchange every sweep, from independent seeds (with a
    shared seed the two chains would stay correlated and the comparison would
    be too lenient).  Also the float32 chain's final configurations measured
    by both kernel sets."""
    from paper_1211_0780_amd.precision import compare as cmp
    res = cmp(64, np.linspace(0.4530, 0.4554, 32), n_sweeps=2000, seeds=(3, 1003))
    gate = bonferroni_z(res["n_compared"])
    print(f"[L=64 fp32 vs fp64] {res['n_compared']} comparisons: max |z| = {res['max_abs_z']:.2f}, "
          f"rms z = {res['rms_z']:.2f}, within 2 sigma {res['frac_within_2sigma']:.3f}, gate {gate:.2f}")
    assert res["max_abs_z"] <= gate
    assert 0.5 <= res["rms_z"] <= 2.0
    for row in res["same_state"]:
        assert row["abs_err_e"] <= 1e-6 and row["abs_err_abs_m"] <= 1e-6


def test_fp32_matches_fp64_over_independent_ladders(gpu):
    """Ensemble form: 32 float32 and 32 float64 ladders (L = 16, 16 replicas
    over [0.44, 0.47], 1 + 8, exchange every sweep), each an independent
    chain, with standard errors from the spread of the ladders rather than
    from binning.  Two families, each at its Bonferroni bound: the four
    ladder averages (e, |m|, m^2, m^4) and the 80 per-beta differences."""
    from paper_1211_0780_amd.precision import compare_ladders
    res = compare_ladders(16, np.linspace(0.44, 0.47, 16), n32=32, n64=32, n_sweeps=2000,
                          seeds=(21, 1021))
    zl = np.array([v["z"] for v in res["ladder_average"].values()])
    gate_l, gate_b = bonferroni_z(zl.size), bonferroni_z(res["n_compared"])
    print(f"[L=16 fp32 vs fp64, 32 + 32 ladders] ladder averages z = {np.round(zl, 2).tolist()} "
          f"(gate {gate_l:.2f}); per beta max |z| {res['max_abs_z']:.2f} (gate {gate_b:.2f}), "
          f"rms {res['rms_z']:.2f}, within 2 sigma {res['frac_within_2sigma']:.3f}")
    assert np.all(np.abs(zl) <= gate_l)
    assert res["max_abs_z"] <= gate_b
    assert 0.5 <= res["rms_z"] <= 2.0


def test_fss_batch_binder_crossing(gpu):
    """The batched finite-size-scaling set: L in {24, 32, 48, 64, 96, 128}, 16 replicas each over
    [0.452, 0.456], one launch per half-sweep for the whole batch, graph
    replayed, autotuned tiles.  Sec. III: U_L curves cross at
    beta_c = 1/2.2019 = 0.45415, inside the ladder: the smallest lattice has
    the larger U_L at the low end of the ladder and the smaller at the top."""
    Ls = [24, 32, 48, 64, 96, 128]
    betas = list(np.linspace(0.452, 0.456, 16))
    s = make(Ls, [betas] * len(Ls), 5)
    s.autotune(1, 10, reps=2)
    n = 3000
    o = gpu_series(s, n, 1, 10, 1)
    U = {}
    for li, L in enumerate(Ls):
        for k in (0, 15):
            p = s.pos_base[li] + k
            U[(L, k)] = binned_ratio(o[:, p, 4], o[:, p, 3], f=lambda a, b: 1 - a / (3 * b * b), discard=0.3)
    for k in (0, 15):
        print("[fss] beta", betas[k], {L: round(U[(L, k)][0], 4) for L in Ls})
    lo_s, lo_b = U[(24, 0)], U[(128, 0)]
    hi_s, hi_b = U[(24, 15)], U[(128, 15)]
    assert lo_s[0] - lo_b[0] > 2 * np.hypot(lo_s[1], lo_b[1])
    assert hi_b[0] - hi_s[0] > 2 * np.hypot(hi_s[1], hi_b[1])
