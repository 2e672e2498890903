"""Write the oracle's long-run statistics of a parallel-tempering ladder.

Runs the CPU FP64 oracle only (oracle.run: sweeps of n_metro Metropolis +
n_or over-relaxation substeps, measurement every sweep, exchange every sweep,
Sec. II and Eq. (3)) as several independent chains from consecutive seeds, one
process per chain, and stores per beta-position the mean and binned error of
e, |m|, m^2, m^4 and U_L = 1 - <m^4>/(3<m^2>^2) (Eqs. (4), (5)) over the
pooled bins of all chains.  The GPU test compares its own chain with these.

    python tests/golden/make_pt_ladder_stats.py --L 32 --R 16 --lo 0.450 --hi 0.458 \
        --n-or 5 --chains 8 --sweeps 1500 --seed0 1002 --out tests/golden/pt_ladder_L32_oracle.json
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from stats_util import binder, bins_mean, bins_ratio, chain_bins  # noqa: E402


def one_chain(job):
    L, betas, seed, n, n_metro, n_or = job
    t0 = time.time()
    _, obs, _, sacc = oracle.run(L, np.array(betas), seed, n, n_metro, n_or, exchange_every=1)
    print(f"chain seed {seed}: {n} sweeps in {time.time() - t0:.0f} s", flush=True)
    return obs, sacc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, required=True)
    ap.add_argument("--R", type=int, required=True)
    ap.add_argument("--lo", type=float, required=True)
    ap.add_argument("--hi", type=float, required=True)
    ap.add_argument("--n-metro", type=int, default=1)
    ap.add_argument("--n-or", type=int, required=True)
    ap.add_argument("--chains", type=int, default=8)
    ap.add_argument("--sweeps", type=int, required=True)
    ap.add_argument("--seed0", type=int, required=True)
    ap.add_argument("--bins", type=int, default=6, help="bins per chain")
    ap.add_argument("--discard", type=float, default=0.2)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    betas = np.linspace(a.lo, a.hi, a.R).tolist()
    jobs = [(a.L, betas, a.seed0 + c, a.sweeps, a.n_metro, a.n_or) for c in range(a.chains)]
    with Pool(min(a.chains, os.cpu_count() or 1)) as pool:
        res = pool.map(one_chain, jobs)
    stats = []
    for k in range(a.R):
        bins = {c: np.concatenate([chain_bins(obs[:, k, c], a.bins, a.discard) for obs, _ in res])
                for c in (1, 2, 3, 4)}
        row = {name: bins_mean(bins[c]) for name, c in (("e", 1), ("abs_m", 2), ("m2", 3), ("m4", 4))}
        row["U_L"] = bins_ratio(bins[4], bins[3], binder)
        stats.append({key: [float(v[0]), float(v[1])] for key, v in row.items()})
    swaps = np.sum([s for _, s in res], axis=0)
    attempts = [sum(((tau % 2) == (p % 2)) for tau in range(a.sweeps)) * a.chains for p in range(a.R - 1)]
    out = {
        "what": "oracle long-run statistics per beta-position (mean, binned error)",
        "command": "python " + " ".join([os.path.relpath(__file__, ROOT)] + sys.argv[1:]),
        "L": a.L, "R": a.R, "betas": betas, "n_metro": a.n_metro, "n_or": a.n_or,
        "exchange_every": 1, "chains": a.chains, "sweeps_per_chain": a.sweeps,
        "seeds": [j[2] for j in jobs], "discard": a.discard, "bins_per_chain": a.bins,
        "swap_acceptance": [float(swaps[p]) / attempts[p] for p in range(a.R - 1)],
        "stats": stats,
    }
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
