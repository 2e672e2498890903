"""Throughput of the 3D XY model hot path on one MI355X.

Workload: L = 160 (N = 4,096,000 sites), 32 parallel-tempering replicas with
beta linearly spaced in [0.4538, 0.4546], float32 angles with float64
reductions, one sweep = 1 checkerboard Metropolis + 10 over-relaxation
substeps, then the per-sweep measurement of every replica and one exchange
step.  A "step" is one such sweep of all 32 replicas (graph-replayed).

Prints one JSON line:
  value     site-updates per second over the timed steps (inputs resident in HBM)
  roofline  the dominant kernel, the fused over-relaxation substep (one launch
            updates both colours), against 8 TB/s HBM at 12 algorithmic bytes
            per site-update (the unfused half-sweep's reads and writes; the
            fused pass moves less, so this fraction can exceed what an unfused
            kernel could reach), timed with HIP events on the simulation's
            stream around each group of consecutive launches of one kind
  cpu_baseline  the CPU FP64 oracle on a bounded sample of the same workload
  fp64_plain    the plain FP64 single-replica kernels at L = 160, for reference,
                and the speed-up of the batch over them
  repeats   the timed region run twice more after the per-kernel timing, with
            the median of the three (value stays the first region's rate)
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin updates/sec at L=160×32 replicas; % HBM roofline; FP32 vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE_F32 = 12.0   # a half-sweep reads N angles, writes N/2: 6N B per N/2 updates
BYTES_PER_UPDATE_F64 = 24.0
FUSED_MIN_BYTES_PER_UPDATE = 8.0  # one pass over both colours: read 4 B and write 4 B per site
SINCOS_AMPLITUDE_DEFICIT = 3.3e-8  # mean 1 - |(cos, sin)| of the hardware sine/cosine (measured on gfx950)

L, R, SEED = 160, 32, 4
BETA_LO, BETA_HI = 0.4538, 0.4546
N_METRO, N_OR = 1, 10
DEFAULT_TILING = "16x20"
DEFAULT_TILING_FUSED = "8x40"


def _oracle_one_sweep(args):
    """One sweep (1 Metropolis + 10 over-relaxation) of one L=160 configuration
    with the CPU oracle; returns (site-updates, seconds)."""
    k, L_, beta, seed, window = args
    import numpy as np
    import oracle
    th = oracle.init(L_, 1, seed, 0)
    t0 = time.perf_counter()
    oracle.sweep(th, L_, np.array([beta]), seed, 0, 0, N_METRO, N_OR, window=window)
    dt = time.perf_counter() - t0
    return (N_METRO + N_OR) * L_ ** 3, dt


def _oracle_run(args):
    """A whole oracle run (sweeps, measurement every sweep, exchange as given)
    on one core; returns (site-updates, seconds)."""
    L_, betas, seed, n, n_metro, n_or, every = args
    import numpy as np
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    oracle.run(L_, np.array(betas), seed, n, n_metro, n_or, exchange_every=every)
    dt = time.perf_counter() - t0
    return (n_metro + n_or) * L_ ** 3 * len(betas) * n, dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(window=0.0):
    """The oracle on the host: all available cores on one sweep of L = 160
    configurations (one process per configuration), then single-core runs,
    side by side, of the L = 8 single-lattice chain in full, 100 sweeps of the
    L = 32 tempering ladder and one sweep of one L = 160 configuration; the
    single-core list ends with the L = 160 sweep time of the median process
    of the first leg."""
    import numpy as np
    import oracle
    oracle.build()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, R))
    betas = np.linspace(BETA_LO, BETA_HI, R)
    jobs = [(k, L, float(betas[k]), SEED, window) for k in range(cores)]
    t0 = time.perf_counter()
    # close + join lets the workers exit on their own: terminating them (what
    # the pool's context manager does) sends signals that profilers running
    # inside each worker may not survive
    pool = mp.get_context("spawn").Pool(cores)
    try:
        res = pool.map(_oracle_one_sweep, jobs)
    finally:
        pool.close()
        pool.join()
    wall = time.perf_counter() - t0
    updates = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    # single core: each run alone in its own process, the two side by side
    singles = [("L=8 single lattice, beta 0.4542, 1 + 1, 10^4 sweeps, measurement every sweep (in full)",
                (8, [0.4542], 1, 10000, 1, 1, 0)),
               ("L=32 ladder, 16 replicas over [0.450, 0.458], 1 + 5, exchange every sweep, 100 sweeps",
                (32, list(np.linspace(0.450, 0.458, 16)), 2, 100, 1, 5, 1)),
               (f"L={L} single configuration, beta 0.4542, one sweep of {N_METRO} + {N_OR} with its measurement",
                (L, [0.4542], SEED, 1, N_METRO, N_OR, 0))]
    pool = mp.get_context("spawn").Pool(len(singles))
    try:
        sres = pool.map(_oracle_run, [a for _, a in singles])
    finally:
        pool.close()
        pool.join()
    single_core = [{"workload": name, "site_updates": u, "seconds": round(t, 2),
                    "ns_per_update": round(1e9 * t / u, 1)} for (name, _), (u, t) in zip(singles, sres)]
    # the L = 160 sweep of one process of the all-cores leg (median process;
    # every core busy meanwhile, so memory bandwidth is shared), beside the
    # same sweep alone on one core above
    per_proc = sorted(r[1] for r in res)[len(res) // 2]
    single_core.append({"workload": f"L={L} single configuration, one sweep of {N_METRO} + {N_OR} "
                                    "(median process of the all-cores leg, every core busy)",
                        "site_updates": res[0][0], "seconds": round(per_proc, 2),
                        "ns_per_update": round(1e9 * per_proc / res[0][0], 1)})
    return {
        "value": updates / busy,
        "unit": "site-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{cores} configurations of L={L} (one process each, one per available core), one "
                  f"sweep of {N_METRO} Metropolis + {N_OR} over-relaxation each, beta in "
                  f"[{BETA_LO}, {BETA_HI}], {proposal_text(window)}; rate over the slowest "
                  "process's sweep time "
                  f"({busy:.1f} s; wall {wall:.1f} s incl. start-up)",
        "host": {"nproc": os.cpu_count(), "cores_available": avail, "cpu_model": cpu_model()},
        "single_core": single_core,
    }


def proposal_text(window):
    if window > 0:
        return f"restricted-window Metropolis proposal theta + {window:g} (U - 1/2)"
    return "uniform Metropolis proposal"


def kernel_source_hash():
    """Hash of the kernel sources and the compiler flags they are built with
    (the traffic counters belong to one build of the kernels)."""
    from paper_1211_0780_amd import build_lib
    h = hashlib.sha256()
    for f in ("xy_kernels.hip", "xy_or2.hip", "xy_or2_kernel.h", "xy_kernel_common.h", "xy_device.h",
              "xy_kernels.h"):
        with open(os.path.join(ROOT, "paper_1211_0780_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(build_lib.flags_signature().encode())
    return h.hexdigest()[:16]


TRAFFIC_FILES = {
    "fused": "traffic_fused_over_relax_L160x32.json",
    "half": "traffic_over_relax_L160x32.json",
    "metro": "traffic_metropolis_L160x32.json",
}


def traffic_path(kind):
    return os.path.join(ROOT, "profiles", TRAFFIC_FILES[kind])


def load_traffic(kernel_hash, kind):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = traffic_path(kind)
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


COPY_BYTES = 1 << 30


def traffic_probe(sim, dev, metro=False):
    """Workload for `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` and the
    other counter passes: a plain device copy of COPY_BYTES (the calibration
    kernel: it must read and write exactly that many bytes), then two
    over-relaxation substeps of the bench configuration (fused: two launches;
    unfused: four) or, with `metro`, two Metropolis substeps (four half-sweep
    launches, each followed by its float64 re-decision launch)."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if metro:
        sim.sweep(1, 0)
        sim.sweep(1, 0)
    else:
        sim.sweep(0, 2)
    torch.cuda.synchronize()
    print("[bench] traffic probe done", file=sys.stderr, flush=True)


def _pmc_rows(path, counter):
    import csv
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            name = r.get("Kernel_Name", "")
            if r.get("Counter_Name") == counter:
                rows.append((name, float(r["Counter_Value"])))
    return rows


def digest_traffic(fetch_csv, write_csv):
    """Scale the profiled kernel's FETCH_SIZE / WRITE_SIZE (the fused
    over-relaxation substep, the over-relaxation half-sweep, or the
    Metropolis half-sweep, whichever the probe ran) by what the same counters
    read for the plain copy of COPY_BYTES, and store the HBM bytes per launch
    together with the kernel source hash."""
    out = {"kernel_source_hash": kernel_source_hash(), "copy_bytes": COPY_BYTES}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _pmc_rows(path, counter)
        copy = [v for n, v in rows if "elementwise" in n or "copy" in n.lower()]
        found = {"fused": [v for n, v in rows if "k_or2_f32" in n],
                 "half": [v for n, v in rows if "k_tile_f32<1," in n],
                 "metro": [v for n, v in rows if "k_tile_f32<0," in n]}
        kind = next((k for k in ("fused", "half", "metro") if found[k]), None)
        if not copy or kind is None:
            raise SystemExit(f"{path}: copy or profiled-kernel dispatches not found")
        vals = found[kind]
        scale = COPY_BYTES / max(copy)
        out[f"{key}_counter_per_launch"] = sum(vals) / len(vals)
        out[f"{key}_copy_counter"] = max(copy)
        out[f"{key}_scale_bytes_per_unit"] = scale
        out[f"{key}_bytes_per_launch"] = out[f"{key}_counter_per_launch"] * scale
    out["hbm_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["kernel"] = kind
    out["algorithmic_bytes_per_launch"] = BYTES_PER_UPDATE_F32 * R * L ** 3 / (1 if kind == "fused" else 2)
    probe = {"fused": "python3 bench.py --traffic-probe", "half": "python3 bench.py --traffic-probe --unfused",
             "metro": "python3 bench.py --metro-probe"}[kind]
    out["commands"] = [
        f"rocprofv3 --pmc {c} -d <dir> -o run --output-format csv -- {probe}"
        for c in ("FETCH_SIZE", "WRITE_SIZE")
    ] + [f"python3 bench.py --digest-traffic <FETCH_SIZE csv> <WRITE_SIZE csv>"]
    path = traffic_path(kind)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=2,
                    help="extra timed regions of --steps sweeps after the first (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=5,
                    help="extra eagerly launched sweeps timed per kernel with HIP events")
    ap.add_argument("--tiling", default=DEFAULT_TILING,
                    help="'TYxTZ' for the tiled half-sweep, or 'auto' to run the autotuner "
                         f"(default {DEFAULT_TILING}: the autotuner's pick for this workload, fixed "
                         "so that timing and counter runs use the same launch shape)")
    ap.add_argument("--tiling-fused", default=DEFAULT_TILING_FUSED,
                    help="'TYxTZ' for the fused over-relaxation kernel (ignored with --tiling auto)")
    ap.add_argument("--window", type=float, default=0.0,
                    help="restricted-window Metropolis proposal theta + W (U - 1/2), 0 < W <= 2 pi "
                         "(default 0: uniform proposal on the circle)")
    ap.add_argument("--unfused", action="store_true",
                    help="run over-relaxation as two half-sweep kernels per substep")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only the workload for HBM counter collection: a plain 1 GiB device "
                         "copy, then one over-relaxation substep of the bench configuration")
    ap.add_argument("--metro-probe", action="store_true",
                    help="like --traffic-probe, with two Metropolis substeps instead of the "
                         "over-relaxation")
    ap.add_argument("--digest-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs of --traffic-probe into "
                         "profiles/traffic_over_relax_L160x32.json")
    args = ap.parse_args()
    if args.digest_traffic:
        digest_traffic(*args.digest_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path "
              "shards by replica across GPUs but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1211_0780_amd.sim import Sim

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    betas = np.linspace(BETA_LO, BETA_HI, R)
    sim = Sim(L, [betas], seed=SEED, prec="fp32", fused_or=not args.unfused)
    N = L ** 3
    if args.tiling == "auto":
        print("[bench] autotune", file=sys.stderr, flush=True)
        tiling = sim.autotune(N_METRO, N_OR, reps=3)[0]
    else:
        ty, tz = (int(v) for v in args.tiling.split("x"))
        sim.set_tiling(0, ty, tz, 0)
        if not args.unfused:
            ty2, tz2 = (int(v) for v in args.tiling_fused.split("x"))
            sim.set_tiling_fused(0, ty2, tz2)
        tiling = sim.get_tiling(0)
    tiling_fused = sim.get_tiling_fused(0)
    if args.window > 0:
        sim.set_proposal_window(args.window)
    if args.traffic_probe or args.metro_probe:
        traffic_probe(sim, dev, metro=args.metro_probe)
        return
    obs = torch.zeros((max(args.steps, args.warmup, 1), R, 5), dtype=torch.float64, device=dev)

    print(f"[bench] warmup {args.warmup} sweeps", file=sys.stderr, flush=True)
    if args.warmup:
        sim.run(args.warmup, N_METRO, N_OR, exchange_every=1, obs=obs)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} sweeps", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    acc0 = sim.metro_accepts()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.run(args.steps, N_METRO, N_OR, exchange_every=1, obs=obs)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acceptance = float((sim.metro_accepts() - acc0).sum()) / (args.steps * N_METRO * N * R)

    # per-kernel device time: HIP events on the sweep's stream around each group
    # of consecutive launches of one kind (group time / launches in the group).
    # These sweeps follow the timed region at once: after even a fraction of a
    # second of idling the GPU clocks down and the first launches run slower.
    tot, cnt = {}, {}
    for _ in range(args.profile_steps):
        ms, n = sim.sweep_profiled(N_METRO, N_OR)
        for k in ms:
            tot[k] = tot.get(k, 0.0) + ms[k]
            cnt[k] = cnt.get(k, 0) + n[k]
    print(f"[bench] per-kernel timing over {args.profile_steps} sweeps done", file=sys.stderr, flush=True)
    # further timed regions of the same length (three in all with the first):
    # their median and spread are reported beside `value`, which stays the
    # first region's rate
    rep_ms = []
    for _ in range(args.repeats):
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        r0.record(stream)
        sim.run(args.steps, N_METRO, N_OR, exchange_every=1, obs=obs)
        r1.record(stream)
        torch.cuda.synchronize()
        rep_ms.append(r0.elapsed_time(r1) / args.steps)
    print(f"[bench] {args.repeats} repeat regions done", file=sys.stderr, flush=True)
    ms_total = ev0.elapsed_time(ev1)
    sec = ms_total / 1e3
    updates = args.steps * (N_METRO + N_OR) * N * R
    value = updates / sec
    o = obs[: args.steps].cpu().numpy()
    if not np.all(np.isfinite(o)):
        raise SystemExit("non-finite observables")
    avg = {k: (tot[k] / cnt[k] if cnt[k] else None) for k in tot}
    overflow = sim.recheck_overflow()
    khash = kernel_source_hash()
    if cnt["over_fused"]:
        kname, kms = "fused over-relaxation substep (k_or2_f32: both colours per launch)", avg["over_fused"]
        bytes_per_launch = BYTES_PER_UPDATE_F32 * R * N
    else:
        kname, kms = "over-relaxation half-sweep (k_tile_f32<kOver>)", avg["over"]
        bytes_per_launch = BYTES_PER_UPDATE_F32 * R * N / 2
    achieved = bytes_per_launch / (kms / 1e3) / 1e9
    traffic = load_traffic(khash, "fused" if cnt["over_fused"] else "half")
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": kname,
        "avg_launch_ms": round(kms, 4),
        "algorithmic_bytes_per_launch": bytes_per_launch,
        "bytes_per_update_counted": BYTES_PER_UPDATE_F32,
        "avg_launch_ms_by_kernel": {k: (round(v, 4) if v is not None else None) for k, v in avg.items()},
        "kernel_source_hash": khash,
    }
    if cnt["over_fused"]:
        # the fused pass reads both colours once and writes both once: its own
        # minimum is 8 B per site-update (16 B per site per launch), so against
        # that the same launch time is a lower fraction
        own_min = FUSED_MIN_BYTES_PER_UPDATE * R * N
        roofline["own_min_bytes_per_update"] = FUSED_MIN_BYTES_PER_UPDATE
        roofline["frac_own_min"] = round(own_min / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if traffic:
        # HBM bytes the counters saw per launch (an upper bound: L2 misses,
        # some of which the Infinity Cache may serve), over the launch time
        roofline["measured_gbs"] = round(traffic / (kms / 1e3) / 1e9, 1)
        roofline["measured_frac"] = round(traffic / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    if cnt["metro"]:
        # the Metropolis half-sweep (one launch per colour; its float64
        # re-decision launch included in the time): 12 B per site-update
        mms = avg["metro"]
        mbytes = BYTES_PER_UPDATE_F32 * R * N / 2
        mtraffic = load_traffic(khash, "metro")
        roofline["metropolis"] = {
            "avg_launch_ms": round(mms, 4),
            "algorithmic_bytes_per_launch": mbytes,
            "achieved": round(mbytes / (mms / 1e3) / 1e9, 1),
            "frac": round(mbytes / (mms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": mtraffic,
            "measured_gbs": round(mtraffic / (mms / 1e3) / 1e9, 1) if mtraffic else None,
        }
    # FP32 against FP64 on the same configurations: the state the timed run
    # left in two replicas, measured by the FP32 kernels and by the FP64
    # kernels of a one-replica FP64 context holding the same angles
    obs32 = sim.measure()
    errs = []
    for k in (0, R - 1):
        s64 = Sim(L, [[float(betas[k])]], seed=SEED, prec="fp64")
        s64.set_angles(sim.get_angles(0, k))
        o64 = s64.measure()[0]
        s64.close()
        errs.append((abs(obs32[k, 1] - o64[1]), abs(obs32[k, 2] - o64[2]), abs(obs32[k, 0] - o64[0]),
                     abs(o64[1])))
    fp32_vs_fp64 = {
        "replicas": [0, R - 1],
        "max_abs_err_e": float(max(e[0] for e in errs)),
        "max_abs_err_abs_m": float(max(e[1] for e in errs)),
        "max_abs_err_E": float(max(e[2] for e in errs)),
        # the hardware sine/cosine return unit vectors 3.3e-8 short on average,
        # which scales every float32 bond term by 1 - 6.5e-8: bound at twice that
        "tolerance_e": 2 * 2 * SINCOS_AMPLITUDE_DEFICIT * float(max(e[3] for e in errs)),
        "tolerance_abs_m": 1e-6,
        "note": "observables of the same configurations from the float32 path (float64 "
                "accumulation) and from the float64 kernels; the energy error is the relative "
                "bias 2 x 3.3e-8 of the hardware sine/cosine amplitude (measured); per-sweep "
                "angle parity with the float64 oracle is 2e-5 rad (float32) and 1e-12 rad "
                "(float64), checked by the tests",
    }
    sim.close()
    del obs
    torch.cuda.synchronize()

    # plain FP64 single-replica kernels at the same L, for reference
    print("[bench] plain FP64 single replica", file=sys.stderr, flush=True)
    s64 = Sim(L, [[0.4542]], seed=SEED, prec="fp64")
    s64.run(2, N_METRO, N_OR, exchange_every=0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n64 = 5
    e0.record(stream)
    s64.run(n64, N_METRO, N_OR, exchange_every=0)
    e1.record(stream)
    torch.cuda.synchronize()
    fp64_rate = n64 * (N_METRO + N_OR) * N / (e0.elapsed_time(e1) / 1e3)
    s64.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.window)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"L={L} periodic cubic XY lattice x {R} parallel-tempering replicas, "
                        f"beta linspace [{BETA_LO}, {BETA_HI}], float32 angles, float64 "
                        f"reductions and exchange, sweep = {N_METRO} Metropolis + {N_OR} "
                        f"over-relaxation, {proposal_text(args.window)}, measurement and "
                        "exchange every sweep, random start",
            "L": L, "replicas": R, "n_metro": N_METRO, "n_or": N_OR, "seed": SEED,
            "proposal_window": args.window,
            "site_updates_per_step": (N_METRO + N_OR) * N * R,
            "tiling": {"ty": tiling[0], "tz": tiling[1], "grid_cap": tiling[2]},
            "tiling_fused": {"ty": tiling_fused[0], "tz": tiling_fused[1]},
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64_plain_single_replica": {
            "value": fp64_rate, "unit": "site-updates/s",
            "note": f"plain one-thread-per-site float64 kernels, L={L}, 1 replica, same sweep",
            "hbm_frac_at_24B": round(fp64_rate * BYTES_PER_UPDATE_F64 / 1e9 / HBM_PEAK_GBS, 4),
        },
        "fp32_vs_fp64": fp32_vs_fp64,
        "repeats": {
            "ms_per_step": [round(x, 5) for x in [ms_total / args.steps] + rep_ms],
            "median_ms_per_step": round(float(np.median([ms_total / args.steps] + rep_ms)), 5),
            "median_value": updates / (float(np.median([ms_total / args.steps] + rep_ms)) * args.steps / 1e3),
            "note": "the timed region run again right after the per-kernel timing; value is the first",
        },
        "speedup_vs_fp64_plain_single_replica": round(value / fp64_rate, 2),
        "metropolis_acceptance": round(acceptance, 5),
        "recheck_overflow": overflow,
        "wall_s_timed": wall,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
