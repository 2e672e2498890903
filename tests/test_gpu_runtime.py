"""GPU runtime behaviour: graph replay equals eager launches, results do not
depend on tiling or persistence, checkpoints resume bit-exactly, batches of
uneven lattices match the oracle lattice by lattice."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import circ, gpu_states

pytestmark = pytest.mark.gpu


def make(L, betas, seed, prec="fp32", start="random", **kw):
    from paper_1211_0780_amd.sim import Sim
    return Sim(L, betas, seed=seed, prec=prec, start=start, **kw)


def set_tiling(s, lattice, ty, tz, grid=0):
    from paper_1211_0780_amd import _capi as C
    C.check(C.lib().xy_set_tiling(s._ctx, lattice, ty, tz, grid), s._ctx)


def all_states(s):
    return [gpu_states(s, l) for l in range(len(s.L))]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_graph_run_equals_eager(gpu, prec):
    betas = list(np.linspace(0.44, 0.47, 4))
    a = make(16, betas, 21, prec)
    b = make(16, betas, 21, prec)
    n = 6
    obs = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    a.run(n, 1, 3, exchange_every=2, obs=obs)
    torch.cuda.synchronize()
    eager = []
    for sidx in range(n):
        b.sweep(1, 3)
        eager.append(b.measure())
        if (sidx + 1) % 2 == 0:
            b.exchange()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.counters() == b.counters()
    assert a.permutation() == b.permutation()
    ob = obs.cpu().numpy()
    ev = np.stack(eager)
    # fused (in-sweep) and standalone measurements visit sites in the same
    # tile order, so energies agree to rounding of the partial sums
    assert np.allclose(ob, ev, rtol=1e-12, atol=1e-9)


def test_results_independent_of_tiling_and_persistence(gpu):
    """Tile shapes and workgroup caps (fewer workgroups than items, each
    taking several in turn) give the same configurations, Metropolis and
    fused over-relaxation."""
    betas = [0.43, 0.45, 0.47]
    ref = None
    for ty, tz, grid in [(24, 24, 0), (4, 6, 0), (2, 3, 0), (8, 8, 5), (6, 2, 7), (24, 1, 3), (24, 24, 15),
                         (24, 24, 3)]:
        s = make(24, betas, 8)
        set_tiling(s, 0, ty, tz, grid)
        for _ in range(3):
            s.sweep(1, 2)
        st = gpu_states(s)
        if ref is None:
            ref = st
        else:
            assert np.array_equal(st, ref), (ty, tz, grid)


def test_checkpoint_resume_is_bit_exact(gpu):
    betas = list(np.linspace(0.44, 0.46, 4))
    a = make([8, 6], [betas, betas[:2]], 31)
    a.run(5, 1, 2, exchange_every=1)
    blob = a.get_state()
    a.run(7, 1, 2, exchange_every=1)
    final = all_states(a), a.permutation(0), a.counters()
    b = make([8, 6], [betas, betas[:2]], 31)
    b.set_state(blob)
    assert b.counters() == (5, 5)
    b.run(7, 1, 2, exchange_every=1)
    assert b.counters() == final[2]
    assert b.permutation(0) == final[1]
    for x, y in zip(all_states(b), final[0]):
        assert np.array_equal(x, y)


def test_set_state_rejects_foreign_blob(gpu):
    from paper_1211_0780_amd._capi import XYError
    a = make(8, [0.4, 0.5], 1)
    b = make(8, [0.4, 0.5], 2)
    with pytest.raises(XYError):
        b.set_state(a.get_state())
    blob = bytearray(a.get_state())
    blob[0] ^= 0xFF
    with pytest.raises(XYError):
        a.set_state(bytes(blob))


def test_uneven_batch_matches_oracle_per_lattice(gpu):
    """Several lattice sizes in one context (one launch per half-sweep covers
    all of them) against the oracle run lattice by lattice, every site of
    each colour of every configuration, from the GPU state (FP32 chain).  A
    decision may differ from the oracle's only within 1e-6 of its threshold."""
    from gpu_util import check_metro_half, colour_mask
    Ls = [6, 10, 12, 8]
    ladders = [list(np.linspace(0.44, 0.46, r)) for r in (2, 3, 1, 2)]
    seed = 5
    s = make(Ls, ladders, seed)
    for sweep in range(2):
        t = s.counters()[0]
        before = all_states(s)
        s.sweep(1, 0)
        after = all_states(s)
        for l, L in enumerate(Ls):
            m0 = colour_mask(L, 0)
            for k in range(len(ladders[l])):
                for c in (0, 1):
                    start = before[l][k] if c == 0 else np.where(m0, after[l][k], before[l][k])
                    got = np.where(m0, after[l][k], before[l][k]) if c == 0 else after[l][k]
                    ref = start.copy()
                    oracle.metro_half(ref, L, ladders[l][k], seed, t, l, k, 0, c)
                    margin = oracle.metro_margin(start, L, ladders[l][k], seed, t, l, k, 0, c)
                    check_metro_half(start, got, ref, margin, L, c, 2e-5)


def test_beta_zero_moments_on_gpu(gpu):
    """beta = 0 exact moments (N independent uniform spins) from a GPU run."""
    L = 8
    N = L ** 3
    s = make(L, [0.0], 3)
    n = 4000
    obs = torch.zeros((n, 1, 5), dtype=torch.float64, device=gpu)
    s.run(n, 1, 2, exchange_every=0, obs=obs)
    o = obs.cpu().numpy()[:, 0]
    e, m2, m4 = o[:, 1], o[:, 3], o[:, 4]
    assert abs(e.mean()) < 4 * np.sqrt(3 / (2 * N) / n)
    assert abs(N * m2.mean() - 1) < 4 / np.sqrt(n)
    assert abs(N * N * m4.mean() - (2 - 1 / N)) < 4 * np.sqrt(20 / n)


def test_autotune_leaves_the_chain_untouched(gpu):
    betas = list(np.linspace(0.44, 0.46, 3))
    a = make(24, betas, 17)
    b = make(24, betas, 17)
    a.run(2, 1, 2, exchange_every=1)
    b.run(2, 1, 2, exchange_every=1)
    before = gpu_states(a), a.metro_accepts(), a.counters(), a.permutation()
    tiles = a.autotune(1, 4, reps=1)
    ty, tz, _ = tiles[0]
    assert 24 % ty == 0 and 24 % tz == 0
    assert np.array_equal(gpu_states(a), before[0])
    assert np.array_equal(a.metro_accepts(), before[1])
    assert a.counters() == before[2] and a.permutation() == before[3]
    a.run(3, 1, 2, exchange_every=1)
    b.run(3, 1, 2, exchange_every=1)
    assert np.array_equal(gpu_states(a), gpu_states(b))


@pytest.mark.parametrize("L,betas,tiles", [
    (16, [0.44, 0.46], None),
    (24, [0.40, 0.45, 0.50], (4, 3)),
    (12, [0.45], (12, 12)),          # one tile per slot: halo rows and planes wrap onto the tile
    (10, [0.3, 0.5], (2, 5)),
    (160, [0.4542], (5, 20)),        # the benchmark lattice
    (160, [0.4542], (16, 20)),       # five columns per thread
    (64, [0.44, 0.46], (32, 8)),     # four columns per thread
    (48, [0.45], (48, 6)),           # one tile per slot in y, five columns per thread
    (160, [0.4542], (8, 40)),        # the benchmark's fused tiles: three columns per thread
    (96, [0.44, 0.46], (12, 8)),     # three columns, 576 of 768 slots filled
    (192, [0.45], (8, 8)),           # three columns, all filled
    (4, [0.44, 0.46], None),         # the smallest lattice: one 4 x 4 tile per slot
    (6, [0.45], None),               # L/2 = 3 sites per row and colour
])
def test_fused_over_relaxation_equals_two_half_sweeps(gpu, L, betas, tiles):
    """The fused substep performs the same float32 operations in the same
    order as the colour-0 and colour-1 half-sweep kernels (which are checked
    against the oracle site by site), so the configurations are bit-identical."""
    from paper_1211_0780_amd.sim import Sim
    a = Sim(L, [betas], seed=19, prec="fp32", fused_or=True)
    b = Sim(L, [betas], seed=19, prec="fp32", fused_or=False)
    if tiles:
        a.set_tiling_fused(0, *tiles)
    for sweep in range(3):
        a.sweep(1, 4)
        b.sweep(1, 4)
        assert np.array_equal(gpu_states(a), gpu_states(b)), sweep
    a.sweep(0, 3)   # odd count: two fused substeps and one pair of half-sweeps
    b.sweep(0, 3)
    assert np.array_equal(gpu_states(a), gpu_states(b))


def test_fused_path_at_its_largest_lattice(gpu):
    """L = 256 is the largest lattice the fused substep takes (its halo rows
    fill one entry per thread); a batch with L = 258 falls back to the
    half-sweep kernels for every substep.  Chains and observables agree with
    the half-sweep path."""
    from paper_1211_0780_amd.sim import Sim
    for Ls in ([256], [258, 8]):
        betas = [[0.45, 0.46]] + [[0.44]] * (len(Ls) - 1)
        a = Sim(Ls, betas, seed=29, prec="fp32", fused_or=True)
        b = Sim(Ls, betas, seed=29, prec="fp32", fused_or=False)
        # which path runs: fused at L = 256, half-sweeps for the batch with L = 258
        if Ls == [256]:
            assert a.get_tiling_fused(0) != (0, 0)
        else:
            assert all(a.get_tiling_fused(l) == (0, 0) for l in range(len(Ls)))
        R = a.R_total
        oa = torch.zeros((2, R, 5), dtype=torch.float64, device=gpu)
        ob = torch.zeros((2, R, 5), dtype=torch.float64, device=gpu)
        a.run(2, 1, 2, exchange_every=1, obs=oa)
        b.run(2, 1, 2, exchange_every=1, obs=ob)
        torch.cuda.synchronize()
        for l in range(len(Ls)):
            assert np.array_equal(gpu_states(a, l), gpu_states(b, l)), Ls
            assert a.permutation(l) == b.permutation(l)
        assert np.allclose(oa.cpu().numpy(), ob.cpu().numpy(), rtol=1e-12, atol=1e-9)
        a.close()
        b.close()


@pytest.mark.parametrize("tiles", [(8, 8), (16, 8), (24, 8), (48, 6)],
                         ids=["1col", "2col", "3col", "5col"])
@pytest.mark.parametrize("with_bonds", [False, True])
def test_fused_measurement_at_every_column_count(gpu, tiles, with_bonds):
    """The measuring fused substep (capped to four wavefronts per SIMD at up
    to three columns per thread when it forms no bond sums) gives the chain,
    exchanges and observables of the half-sweep path at every column count."""
    from paper_1211_0780_amd.sim import Sim
    L, betas, n = 48, [0.44, 0.45, 0.46], 3
    a = Sim(L, [betas], seed=23, prec="fp32", fused_or=True)
    b = Sim(L, [betas], seed=23, prec="fp32", fused_or=False)
    a.set_tiling_fused(0, *tiles)
    oa = torch.zeros((n, 3, 5), dtype=torch.float64, device=gpu)
    ob = torch.zeros((n, 3, 5), dtype=torch.float64, device=gpu)
    ba = torch.zeros((n, 3, 6), dtype=torch.float64, device=gpu) if with_bonds else None
    bb = torch.zeros((n, 3, 6), dtype=torch.float64, device=gpu) if with_bonds else None
    a.run(n, 1, 2, exchange_every=1, obs=oa, bonds=ba)
    b.run(n, 1, 2, exchange_every=1, obs=ob, bonds=bb)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.permutation() == b.permutation()
    # the partial sums group sites differently: equal up to float64 rounding
    assert np.allclose(oa.cpu().numpy(), ob.cpu().numpy(), rtol=1e-12, atol=1e-9)
    if with_bonds:
        assert np.allclose(ba.cpu().numpy(), bb.cpu().numpy(), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("prec,fused", [("fp32", True), ("fp32", False), ("fp64", False)])
def test_measurement_without_bond_sums(gpu, prec, fused):
    """A run that records no bond sums skips them in the measurement; the
    chain, the observables and the exchanges stay those of a run that
    records them."""
    from paper_1211_0780_amd.sim import Sim
    betas = list(np.linspace(0.44, 0.46, 4))
    a = Sim([12, 10], [betas, betas[:3]], seed=8, prec=prec, fused_or=fused)
    b = Sim([12, 10], [betas, betas[:3]], seed=8, prec=prec, fused_or=fused)
    n = 4
    oa = torch.zeros((n, 7, 5), dtype=torch.float64, device=gpu)
    ob = torch.zeros((n, 7, 5), dtype=torch.float64, device=gpu)
    bb = torch.zeros((n, 7, 6), dtype=torch.float64, device=gpu)
    a.run(n, 1, 4, exchange_every=1, obs=oa)
    b.run(n, 1, 4, exchange_every=1, obs=ob, bonds=bb)
    torch.cuda.synchronize()
    for l in range(2):
        assert np.array_equal(gpu_states(a, l), gpu_states(b, l))
        assert a.permutation(l) == b.permutation(l)
    assert np.array_equal(oa.cpu().numpy(), ob.cpu().numpy())
    assert np.all(bb.cpu().numpy()[:, :, :3] != 0.0)


@pytest.mark.parametrize("exchange_every", [0, 1])
def test_batched_graph_replay_matches_single_sweeps(gpu, exchange_every):
    """A long run replays graphs of several sweeps plus single-sweep graphs
    for the remainder; its chain, permutation, counters and observable ring
    equal those of one-sweep runs."""
    betas = list(np.linspace(0.44, 0.46, 4))
    n = 11
    a = make(10, betas, 21)
    b = make(10, betas, 21)
    oa = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    ob = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    a.run(n, 1, 2, exchange_every=exchange_every, obs=oa)
    for s in range(n):
        b.run(1, 1, 2, exchange_every=exchange_every, obs=ob[s:s + 1])
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.permutation() == b.permutation()
    assert a.counters() == b.counters() == (n, n * exchange_every)
    assert np.array_equal(oa.cpu().numpy(), ob.cpu().numpy())


def test_many_rings_release_old_graphs(gpu):
    """A fresh observable ring on every call captures new graphs; past the
    context's limit the oldest are released, and the chain is unaffected."""
    betas = [0.44, 0.45, 0.46]
    n = 40
    a = make(8, betas, 3)
    b = make(8, betas, 3)
    ob = torch.zeros((n, 3, 5), dtype=torch.float64, device=gpu)
    b.run(n, 1, 1, exchange_every=1, obs=ob)
    rings = []
    for _ in range(n):
        rings.append(torch.zeros((1, 3, 5), dtype=torch.float64, device=gpu))
        a.run(1, 1, 1, exchange_every=1, obs=rings[-1])
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.permutation() == b.permutation()
    assert np.array_equal(torch.cat(rings).cpu().numpy(), ob.cpu().numpy())


def test_metropolis_only_sweeps_measure_the_final_state(gpu):
    """With no over-relaxation the sweep ends on a Metropolis half-sweep whose
    near-threshold decisions are re-taken after it; the loop then measures
    the final configuration with the standalone pass, exactly as an eager
    sweep + measure + exchange does."""
    betas = list(np.linspace(0.44, 0.46, 4))
    n = 5
    a = make(12, betas, 17)
    b = make(12, betas, 17)
    oa = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    a.run(n, 1, 0, exchange_every=1, obs=oa)
    torch.cuda.synchronize()
    ob = []
    for _ in range(n):
        b.sweep(1, 0)
        ob.append(b.measure())
        b.exchange()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.permutation() == b.permutation()
    assert np.array_equal(oa.cpu().numpy(), np.stack(ob))


def test_fused_measurement_equals_half_sweep_measurement(gpu):
    from paper_1211_0780_amd.sim import Sim
    betas = list(np.linspace(0.44, 0.46, 4))
    a = Sim(16, [betas], seed=4, prec="fp32", fused_or=True)
    b = Sim(16, [betas], seed=4, prec="fp32", fused_or=False)
    n = 5
    oa = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    ob = torch.zeros((n, 4, 5), dtype=torch.float64, device=gpu)
    ba = torch.zeros((n, 4, 6), dtype=torch.float64, device=gpu)
    bb = torch.zeros((n, 4, 6), dtype=torch.float64, device=gpu)
    a.run(n, 1, 4, exchange_every=1, obs=oa, bonds=ba)
    b.run(n, 1, 4, exchange_every=1, obs=ob, bonds=bb)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.permutation() == b.permutation()
    assert np.allclose(oa.cpu().numpy(), ob.cpu().numpy(), rtol=1e-12, atol=1e-9)
    assert np.allclose(ba.cpu().numpy(), bb.cpu().numpy(), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("fused", [True, False])
def test_profiled_sweep_equals_sweep(gpu, fused):
    """The profiling variant launches the same kernels in the same order as
    xy_sweep and reports one launch count per kernel group."""
    from paper_1211_0780_amd.sim import Sim
    betas = [0.44, 0.45, 0.46]
    a = Sim(12, [betas], seed=23, prec="fp32", fused_or=fused)
    b = Sim(12, [betas], seed=23, prec="fp32", fused_or=fused)
    for _ in range(2):
        ms, n = a.sweep_profiled(1, 5)
        b.sweep(1, 5)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert a.counters() == b.counters()
    nf = 4 if fused else 0
    assert n == {"metro": 2, "over": 2 * (5 - nf), "over_fused": nf, "other": 1}
    assert all(ms[k] > 0 for k in n if n[k]) and all(ms[k] == 0 for k in n if not n[k])


def test_fused_batch_with_mixed_tiles_equals_half_sweeps(gpu):
    """One fused launch covers every lattice of a batch: the largest tile sets
    the columns per thread of the launch, also for lattices with small tiles."""
    from paper_1211_0780_amd.sim import Sim
    L = [64, 16, 10]
    betas = [[0.44, 0.46], [0.45], [0.40, 0.50]]
    a = Sim(L, betas, seed=29, prec="fp32", fused_or=True)
    b = Sim(L, betas, seed=29, prec="fp32", fused_or=False)
    a.set_tiling_fused(0, 32, 8)
    for sweep in range(2):
        a.sweep(1, 4)
        b.sweep(1, 4)
        torch.cuda.synchronize()
        assert torch.equal(a.angles, b.angles), sweep


def test_lattice_chain_does_not_depend_on_the_rest_of_the_batch(gpu):
    """The counters carry the lattice index, so a lattice's chain is the same
    alone and as the first lattice of a batch, exchange and fused launches
    included (the other lattices only share the launches)."""
    import torch
    betas = [0.44, 0.45, 0.46]
    alone = make([32], [betas], 41)
    batch = make([32, 16, 24], [betas, [0.3, 0.5], [0.45]], 41)
    obs_a = torch.zeros((4, 3, 5), dtype=torch.float64, device=gpu)
    obs_b = torch.zeros((4, 6, 5), dtype=torch.float64, device=gpu)
    alone.run(4, 1, 5, exchange_every=1, obs=obs_a)
    batch.run(4, 1, 5, exchange_every=1, obs=obs_b)
    torch.cuda.synchronize()
    assert np.array_equal(gpu_states(alone, 0), gpu_states(batch, 0))
    assert alone.permutation()[:3] == batch.permutation()[:3]
    assert np.allclose(obs_a.cpu().numpy(), obs_b[:, :3].cpu().numpy(), rtol=1e-12, atol=1e-9)


def test_run_reports_non_finite_state(gpu):
    """A non-finite angle written by the caller into its own buffer (a failure
    forced from the host) makes the next loop's measurement non-finite; the
    loop itself does not wait, and the following xy_run reports
    XY_ERR_STATE once it can see the loop has finished.  xy_measure into host
    memory reports it as well."""
    from paper_1211_0780_amd import _capi as C
    s = make(8, [0.44, 0.45], 31)
    s.run(2, 1, 2, exchange_every=1)
    torch.cuda.synchronize()
    s.run(1, 1, 2, exchange_every=1)          # a clean state reports nothing
    torch.cuda.synchronize()
    s.angles.view(torch.float32)[7] = float("nan")
    torch.cuda.synchronize()
    s.run(2, 1, 2, exchange_every=1)          # asynchronous: returns at once
    torch.cuda.synchronize()
    with pytest.raises(C.XYError) as e:
        s.run(1, 1, 2, exchange_every=1)
    assert e.value.status == C.XY_ERR_STATE
    with pytest.raises(C.XYError) as e:
        s.measure()
    assert e.value.status == C.XY_ERR_STATE
    s.close()


def test_autotuned_schedule_gives_the_same_chain(gpu):
    """Whatever tiles, over-relaxation schedule (fused pass or two half-sweep
    launches) and workgroup cap the autotuner picks for an uneven batch, the
    chain is bit-identical to the default launches; setting a fused tile
    selects the fused schedule again."""
    ladders = [[0.44, 0.45, 0.46], [0.43, 0.47]]
    a = make([24, 16], ladders, 41)
    b = make([24, 16], ladders, 41)
    a.autotune(1, 4, reps=1)
    tuned = [a.get_tiling_fused(l) for l in range(2)]
    oa = torch.zeros((3, 5, 5), dtype=torch.float64, device=gpu)
    ob = torch.zeros((3, 5, 5), dtype=torch.float64, device=gpu)
    a.run(3, 1, 4, exchange_every=1, obs=oa)
    b.run(3, 1, 4, exchange_every=1, obs=ob)
    torch.cuda.synchronize()
    for l in range(2):
        assert np.array_equal(gpu_states(a, l), gpu_states(b, l)), (l, tuned)
        assert a.permutation(l) == b.permutation(l)
    # the reduction order follows the tiles: energies agree to float64 rounding
    assert np.allclose(oa.cpu().numpy(), ob.cpu().numpy(), rtol=1e-12, atol=1e-9)
    a.set_tiling_fused(0, 4, 8)
    assert a.get_tiling_fused(0) == (4, 8) and a.get_tiling_fused(1) != (0, 0)
    print(f"[autotune] fused tiles after tuning {tuned}, grid cap {a.get_tiling(0)[2]}")
    a.close()
    b.close()


def test_run_rings_in_pinned_host_memory(gpu):
    """The loop writes its observable and bond rings straight into pinned
    host memory (the GPU reaches it through its mapped address): the same
    values as device rings from the same start, and the same chain."""
    betas = list(np.linspace(0.44, 0.46, 3))
    a = make(8, betas, 41)
    b = make(8, betas, 41)
    n = 6
    od = torch.zeros((n, 3, 5), dtype=torch.float64, device=gpu)
    bd = torch.zeros((n, 3, 6), dtype=torch.float64, device=gpu)
    oh = torch.zeros((n, 3, 5), dtype=torch.float64, pin_memory=True)
    bh = torch.zeros((n, 3, 6), dtype=torch.float64, pin_memory=True)
    a.run(n, 1, 2, exchange_every=1, obs=od, bonds=bd)
    b.run(n, 1, 2, exchange_every=1, obs=oh, bonds=bh)
    torch.cuda.synchronize()
    assert np.array_equal(od.cpu().numpy(), oh.numpy())
    assert np.array_equal(bd.cpu().numpy(), bh.numpy())
    assert np.array_equal(gpu_states(a), gpu_states(b))
    assert np.all(oh.numpy()[:, :, 0] < 0)
    # xy_measure and xy_get_bond_sums with a pinned host destination and the
    # on-device flag (asynchronous, written by the device)
    import ctypes
    from paper_1211_0780_amd import _capi as C
    mo = torch.zeros((3, 5), dtype=torch.float64, pin_memory=True)
    mb = torch.zeros((3, 6), dtype=torch.float64, pin_memory=True)
    C.check(C.lib().xy_measure(b._ctx, ctypes.c_void_p(mo.data_ptr()), 1), b._ctx)
    C.check(C.lib().xy_get_bond_sums(b._ctx, ctypes.c_void_p(mb.data_ptr()), 1), b._ctx)
    torch.cuda.synchronize()
    assert np.allclose(mo.numpy(), a.measure(), rtol=1e-12, atol=1e-9)
    assert np.allclose(mb.numpy(), a.bond_sums(), rtol=1e-12, atol=1e-9)


def _allocation_bytes_after(ptr):
    """Bytes from ptr to the end of its HIP allocation (None if not reported)."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    base, size = ctypes.c_void_p(), ctypes.c_size_t()
    if hip.hipMemGetAddressRange(ctypes.byref(base), ctypes.byref(size), ctypes.c_void_p(ptr)) != 0:
        hip.hipGetLastError()
        return None
    return base.value + size.value - ptr


def test_buffers_the_gpu_cannot_write_are_rejected(gpu):
    """Pageable host memory where the GPU writes (the loop's rings, xy_measure
    and xy_get_bond_sums with their on-device flag) and a ring shorter than
    the run (its allocation ends first) are refused with XY_ERR_ARG before
    anything is enqueued: the chain and the counters do not move."""
    import ctypes
    from paper_1211_0780_amd import _capi as C
    s = make(8, [0.44, 0.46], 5)
    before = gpu_states(s)
    counters = s.counters()
    host = np.zeros(64 * 2 * 6)
    p = host.ctypes.data_as(ctypes.c_void_p)
    assert C.lib().xy_run_ex(s._ctx, 8, 1, 1, 1, p, None) == C.XY_ERR_ARG
    assert C.lib().xy_run_ex(s._ctx, 8, 1, 1, 1, None, p) == C.XY_ERR_ARG
    assert C.lib().xy_measure(s._ctx, p, 1) == C.XY_ERR_ARG
    assert C.lib().xy_get_bond_sums(s._ctx, p, 1) == C.XY_ERR_ARG
    # a pinned ring whose allocation ends one sweep's records too early
    ring = torch.zeros(16, dtype=torch.float64, pin_memory=True)
    room = _allocation_bytes_after(ring.data_ptr())
    if room is None:
        pytest.skip("the allocation range of pinned host memory is not reported")
    n_fit = room // (5 * 2 * 8)
    assert C.lib().xy_run_ex(s._ctx, int(n_fit + 1), 1, 1, 1, ctypes.c_void_p(ring.data_ptr()), None) == C.XY_ERR_ARG
    assert "smaller than" in C.lib().xy_last_error(s._ctx).decode()
    assert s.counters() == counters
    assert np.array_equal(gpu_states(s), before)
