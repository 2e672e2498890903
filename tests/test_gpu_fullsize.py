"""Parity at the benchmark's full size (L = 160 x 32 replicas, in the launch
shape bench.py times) and at the largest lattice the library accepts
(L = 1024), through the C ABI.

Full size: whole replicas are read back and every site of a half-sweep is
compared with the oracle's half-sweep from the same state.  L = 1024 (4.3 GB
of float32 angles): sampled sites against the closed forms of the random
start and of a beta = 0 Metropolis sweep (bit-exact), and energy
conservation of over-relaxation (a property that holds at any size).
"""
import numpy as np
import pytest

import oracle
import oracle.philox_py as P
from gpu_util import circ, colour_mask, e_tol_fp32, field_numpy

pytestmark = pytest.mark.gpu

L_BENCH, R_BENCH = 160, 32
BENCH_TILING, BENCH_TILING_FUSED = (16, 20), (8, 40)


def make(L, betas, seed, prec="fp32", start="random"):
    from paper_1211_0780_amd.sim import Sim
    return Sim(L, betas, seed=seed, prec=prec, start=start)


@pytest.fixture(scope="module")
def bench_sim(gpu):
    betas = np.linspace(0.4538, 0.4546, R_BENCH)
    s = make(L_BENCH, [betas], 4)
    s.set_tiling(0, *BENCH_TILING, 0)   # the launch shapes bench.py times
    s.set_tiling_fused(0, *BENCH_TILING_FUSED)
    yield s, betas
    s.close()


def test_full_size_fused_sweep_equals_half_sweeps(bench_sim):
    """A whole sweep (1 + 10) in the benchmark's launch shapes, with the ten
    over-relaxation substeps as five fused launches, leaves bit-for-bit the
    configuration that the half-sweep kernels (checked site by site against
    the oracle above) produce from the same state."""
    import torch
    from paper_1211_0780_amd.sim import Sim
    s, betas = bench_sim
    ref = Sim(L_BENCH, [betas], seed=4, prec="fp32", fused_or=False)
    ref.set_tiling(0, *BENCH_TILING, 0)
    ref.set_state(s.get_state())
    s.sweep(1, 10)
    ref.sweep(1, 10)
    torch.cuda.synchronize()
    assert torch.equal(s.angles, ref.angles)
    assert s.counters() == ref.counters()
    ref.close()


def test_full_size_fused_measurement(bench_sim):
    """The measurement fused into the last over-relaxation launch of a
    graph-replayed sweep (the benchmark's path) against the standalone
    measurement kernel on the same configurations and against the oracle."""
    import torch
    s, betas = bench_sim
    N = L_BENCH ** 3
    obs = torch.zeros((1, R_BENCH, 5), dtype=torch.float64, device="cuda")
    s.run(1, 1, 10, exchange_every=0, obs=obs)
    torch.cuda.synchronize()
    fused = obs[0].cpu().numpy()
    standalone = s.measure()
    assert np.allclose(fused, standalone, rtol=1e-12, atol=1e-6)
    for k in (0, R_BENCH - 1):
        ref = oracle.measure(s.get_angles(0, k), L_BENCH)
        assert abs(fused[k, 0] - ref[0]) <= e_tol_fp32(ref[0], N)
        assert abs(fused[k, 2] - ref[2]) <= 1e-6


def test_full_size_over_relaxation_every_site(bench_sim):
    s, betas = bench_sim
    L = L_BENCH
    starts = {k: s.get_angles(0, k) for k in (0, R_BENCH - 1)}
    s.sweep(0, 1)
    m0 = colour_mask(L, 0)
    for k, before in starts.items():
        after = s.get_angles(0, k)
        ref = before.copy()
        oracle.or_half(ref, L, 0)
        hx, hy = field_numpy(before, L)
        bound = np.maximum(2e-5, 16 * 2.0 ** -24 * 6 / np.maximum(np.hypot(hx, hy), 1e-30))
        assert np.all((circ(after, ref) <= bound)[m0])
        mid = before.copy()
        mid[m0] = after[m0]
        ref = mid.copy()
        oracle.or_half(ref, L, 1)
        hx, hy = field_numpy(mid, L)
        bound = np.maximum(2e-5, 16 * 2.0 ** -24 * 6 / np.maximum(np.hypot(hx, hy), 1e-30))
        assert np.all((circ(after, ref) <= bound)[~m0])


def test_full_size_metropolis_every_site(bench_sim):
    """One Metropolis substep at full size: every site of both colours of four
    configurations (beta-positions 0, 5, 17, 31) against the oracle's
    half-sweeps from the GPU's own states; colour 1 runs after the float64
    re-decision of colour 0.  Decisions may differ only within 1e-6 of the
    threshold (proposals are exact in turns, so agreeing sites match to the
    float64 rounding of 2 pi u)."""
    from gpu_util import check_metro_half
    s, betas = bench_sim
    L, seed = L_BENCH, 4
    t = s.counters()[0]
    ks = (0, 5, 17, 31)
    before = {k: s.get_angles(0, k) for k in ks}
    acc0 = s.metro_accepts()
    s.sweep(1, 0)
    acc1 = s.metro_accepts()
    m0 = colour_mask(L, 0)
    flips = 0
    for k in ks:
        after = s.get_angles(0, k)
        n_ref = 0
        for c in (0, 1):
            start = before[k] if c == 0 else np.where(m0, after, before[k])
            got = np.where(m0, after, before[k]) if c == 0 else after
            ref = start.copy()
            n_ref += oracle.metro_half(ref, L, betas[k], seed, t, 0, k, 0, c)
            margin = oracle.metro_margin(start, L, betas[k], seed, t, 0, k, 0, c)
            nf = check_metro_half(start, got, ref, margin, L, c, 1e-6)
            flips += nf
        assert abs(int(acc1[k] - acc0[k]) - n_ref) <= flips
    print(f"[full-size metropolis] {len(ks)} configurations, both colours: {flips} near-threshold flips")
    assert flips <= 5
    assert s.recheck_overflow() == 0


def test_full_size_windowed_metropolis_every_site(gpu):
    """The restricted-window proposal theta' = theta + 2.0 (U - 1/2) (the
    second Metropolis workload, timed by bench.py --window 2.0) at full size
    in the benchmark's tiling: one Metropolis substep, every site of both
    colours of beta-positions 0 and 31 against the oracle's half-sweeps from
    the GPU's own states, decisions differing only within 1e-6 of the
    threshold."""
    from gpu_util import check_metro_half
    L, seed, w = L_BENCH, 6, 2.0
    betas = np.linspace(0.4538, 0.4546, R_BENCH)
    s = make(L, [betas], seed)
    s.set_tiling(0, *BENCH_TILING, 0)
    s.set_tiling_fused(0, *BENCH_TILING_FUSED)
    s.set_proposal_window(w)
    s.sweep(1, 2)
    t = s.counters()[0]
    ks = (0, R_BENCH - 1)
    before = {k: s.get_angles(0, k) for k in ks}
    acc0 = s.metro_accepts()
    s.sweep(1, 0)
    acc1 = s.metro_accepts()
    m0 = colour_mask(L, 0)
    flips, n_acc = 0, 0
    for k in ks:
        after = s.get_angles(0, k)
        n_ref = 0
        for c in (0, 1):
            start = before[k] if c == 0 else np.where(m0, after, before[k])
            got = np.where(m0, after, before[k]) if c == 0 else after
            ref = start.copy()
            n_ref += oracle.metro_half(ref, L, betas[k], seed, t, 0, k, 0, c, window=w)
            margin = oracle.metro_margin(start, L, betas[k], seed, t, 0, k, 0, c, window=w)
            flips += check_metro_half(start, got, ref, margin, L, c, 2e-5)
        assert abs(int(acc1[k] - acc0[k]) - n_ref) <= flips
        n_acc += n_ref
    print(f"[full-size windowed metropolis] acceptance {n_acc / (len(ks) * L ** 3):.3f}, "
          f"{flips} near-threshold flips")
    assert flips <= 5
    assert s.recheck_overflow() == 0
    s.close()


def test_full_size_bond_sums(bench_sim):
    """The bond sums behind Eq. (6) at full size: one graph-replayed sweep
    with a bond ring, so the last over-relaxation launch is the fused
    measuring kernel that also forms the sums, against the standalone bond
    kernel on the same configurations and against the oracle's sums."""
    import torch
    s, betas = bench_sim
    N = L_BENCH ** 3
    obs = torch.zeros((1, R_BENCH, 5), dtype=torch.float64, device="cuda")
    bonds = torch.zeros((1, R_BENCH, 6), dtype=torch.float64, device="cuda")
    s.run(1, 1, 10, exchange_every=0, obs=obs, bonds=bonds)
    torch.cuda.synchronize()
    fused = bonds[0].cpu().numpy()
    assert np.allclose(fused, s.bond_sums(), rtol=1e-12, atol=1e-6)
    for k in (0, R_BENCH - 1):
        ref = oracle.bond_sums(s.get_angles(0, k), L_BENCH)
        assert np.allclose(fused[k], ref, rtol=0, atol=2e-6 * N), (fused[k], ref)
    # the energy of the same launch is the negative sum of the C terms
    assert np.allclose(obs[0, :, 0].cpu().numpy(), -fused[:, :3].sum(axis=1), rtol=0, atol=2e-6 * N)


def test_full_size_measurement(bench_sim):
    s, betas = bench_sim
    obs = s.measure()
    N = L_BENCH ** 3
    for k in (0, 17):
        ref = oracle.measure(s.get_angles(0, k), L_BENCH)
        assert abs(obs[k, 0] - ref[0]) <= e_tol_fp32(ref[0], N)
        assert abs(obs[k, 2] - ref[2]) <= 1e-6


def test_max_lattice_sampled(gpu):
    import torch
    L, seed = 1024, 77
    N = L ** 3
    if torch.cuda.get_device_properties(0).total_memory < 16 * N:
        pytest.skip("device too small for L = 1024")
    s = make(L, [[0.0]], seed)
    rng = np.random.default_rng(1)
    sites = np.unique(np.concatenate([rng.integers(0, N, 4000), [0, N - 1, L - 1, N - L]]))
    key = P.key_of(seed)
    got = s.get_sites(sites)
    want = np.array([2 * np.pi * P.uniform(P.philox4x32_10(P.counter(int(i), 0, 0, 0, P.PHASE_INIT, 0), key)[0])
                     for i in sites])
    assert np.array_equal(got, want)
    s.sweep(1, 0)
    got = s.get_sites(sites)
    want = np.array([2 * np.pi * P.uniform(P.metro_words(int(i), L, 0, 0, 0, 0, key)[0])
                     for i in sites])
    assert np.array_equal(got, want)
    E0 = s.measure()[0, 0]
    s.sweep(0, 2)
    E1 = s.measure()[0, 0]
    assert abs(E1 - E0) <= 1e-7 * N
    s.close()


def test_full_size_fp64_half_sweeps_match_oracle(gpu):
    """The plain FP64 kernels (the single-replica reference the benchmark
    reports) at L = 160, every site against the oracle, one half-sweep at a
    time from the same state: Metropolis exactly (same decisions, same
    proposals), over-relaxation within max(1e-12, 16 * 6 * 2^-53 / |h|) rad.
    Whole sweeps are not compared at this size: over-relaxation amplifies
    rounding differences between two correct FP64 evaluations roughly tenfold
    per substep, so after ten substeps a few sites differ by ~1e-3 rad."""
    L, beta, seed = L_BENCH, 0.4542, 4
    s = make(L, [[beta]], seed, prec="fp64")
    m0 = colour_mask(L, 0)
    before = s.get_angles(0, 0)
    s.sweep(1, 0)
    after = s.get_angles(0, 0)
    ref = before.copy()
    acc0 = oracle.metro_half(ref, L, beta, seed, 0, 0, 0, 0, 0)
    acc1 = oracle.metro_half(ref, L, beta, seed, 0, 0, 0, 0, 1)
    assert np.max(circ(after, ref)) <= 1e-12
    assert s.metro_accepts()[0] == acc0 + acc1
    before = after
    s.sweep(0, 1)
    after = s.get_angles(0, 0)
    for colour, base in ((0, before), (1, np.where(m0, after, before))):
        ref = base.copy()
        oracle.or_half(ref, L, colour)
        hx, hy = field_numpy(base, L)
        bound = np.maximum(1e-12, 16 * 6 * 2.0 ** -53 / np.maximum(np.hypot(hx, hy), 1e-300))
        mask = m0 if colour == 0 else ~m0
        assert np.all((circ(after, ref) <= bound)[mask]), colour
    s.close()
