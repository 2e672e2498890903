"""Float32 against float64 kernels on one beta-ladder (host driver over the C ABI).

Runs the same ladder twice, once with the float32 path (float32 angles and
spin arithmetic, float64 near-threshold re-decision and float64 reductions)
and once with the all-float64 kernels, from independent seeds, and reports
per beta the difference of the long-run averages of e, |m|, m^2, m^4 and
U_L (Eqs. (4), (5)) in units of their combined binning error.  Both chains
sample the same Boltzmann law, so the differences should look like draws
from a unit normal.  Same-configuration errors of the reductions are added
by loading the float32 chain's final configurations into a float64 context.

    python -m paper_1211_0780_amd.precision --sweeps 10000
"""
import argparse
import json
import sys

import numpy as np

from . import analysis as A

NAMES = ("e", "|m|", "m2", "m4", "U_L")


def _series(sim, n_sweeps, n_metro, n_or):
    import torch
    obs = torch.zeros((n_sweeps, sim.R_total, 5), dtype=torch.float64, device=sim.device)
    sim.run(n_sweeps, n_metro, n_or, exchange_every=1, obs=obs)
    torch.cuda.synchronize()
    return obs.cpu().numpy()


def _summary(o, discard):
    rows = []
    for p in range(o.shape[1]):
        row = [A.binned(o[:, p, c], discard=discard) for c in (1, 2, 3, 4)]
        row.append(A.binder(o[:, p, 3], o[:, p, 4], discard=discard))
        rows.append(row)
    return rows


def compare(L, betas, n_sweeps=10000, n_metro=1, n_or=8, seeds=(3, 1003), discard=0.2):
    from .sim import Sim

    s32 = Sim(L, [betas], seed=seeds[0], prec="fp32")
    s64 = Sim(L, [betas], seed=seeds[1], prec="fp64")
    o32 = _series(s32, n_sweeps, n_metro, n_or)
    o64 = _series(s64, n_sweeps, n_metro, n_or)
    a, b = _summary(o32, discard), _summary(o64, discard)
    per_beta, zs = [], []
    for k, beta in enumerate(betas):
        row = {"beta": float(beta)}
        for name, (ma, ea), (mb, eb) in zip(NAMES, a[k], b[k]):
            z = (ma - mb) / np.hypot(ea, eb)
            zs.append(z)
            row[name] = {"fp32": ma, "fp64": mb, "err": float(np.hypot(ea, eb)), "z": float(z)}
        per_beta.append(row)
    # the float32 chain's final configurations, measured by both kernel sets
    same = []
    obs32 = s32.measure()
    for k in (0, len(betas) - 1):
        ref = Sim(L, [[float(betas[k])]], seed=seeds[1], prec="fp64")
        ref.set_angles(s32.get_angles(0, k))
        o = ref.measure()[0]
        ref.close()
        same.append({"beta_pos": k, "abs_err_e": float(abs(obs32[k, 1] - o[1])),
                     "abs_err_abs_m": float(abs(obs32[k, 2] - o[2]))})
    s32.close()
    s64.close()
    zs = np.array(zs)
    return {"L": L, "betas": [float(x) for x in betas], "n_sweeps": n_sweeps, "n_metro": n_metro,
            "n_or": n_or, "seeds": list(seeds), "discard": discard,
            "max_abs_z": float(np.max(np.abs(zs))), "mean_z": float(np.mean(zs)),
            "rms_z": float(np.sqrt(np.mean(zs ** 2))), "n_compared": int(zs.size),
            "frac_within_2sigma": float(np.mean(np.abs(zs) <= 2.0)),
            "same_state": same, "per_beta": per_beta}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--beta", type=float, nargs=2, default=[0.4530, 0.4554])
    ap.add_argument("--replicas", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=10000)
    ap.add_argument("--n-or", type=int, default=8)
    ap.add_argument("--seeds", type=int, nargs=2, default=[3, 1003])
    args = ap.parse_args(argv)
    betas = np.linspace(args.beta[0], args.beta[1], args.replicas)
    res = compare(args.L, betas, n_sweeps=args.sweeps, n_or=args.n_or, seeds=tuple(args.seeds))
    json.dump(res, sys.stdout)
    print()


if __name__ == "__main__":
    main()
