"""Float32 against float64 kernels on a beta-ladder (host driver over the C ABI).

Runs the same ladder twice, once with the float32 path (float32 angles and
spin arithmetic, float64 near-threshold re-decision and float64 reductions)
and once with the all-float64 kernels, from independent seeds, and reports
per beta the difference of the long-run averages of e, |m|, m^2, m^4 and
U_L (Eqs. (4), (5)) in units of their combined binning error.  Both chains
sample the same Boltzmann law, so the differences should look like draws
from a unit normal.  Same-configuration errors of the reductions are added
by loading the float32 chain's final configurations into a float64 context.

    python -m paper_1211_0780_amd.precision --sweeps 10000

The betas of one exchange-coupled ladder move together and its binning
errors rest on the autocorrelation estimate, so one ladder pair is only a
few independent comparisons.  With --ladders K32 K64 the study instead runs
K32 float32 and K64 float64 ladders, each an independent chain (one batch
per precision, one launch per half-sweep for the whole batch), and compares
the ensemble means with standard errors from the spread of the ladders,
which assume nothing about autocorrelation:

    python -m paper_1211_0780_amd.precision --sweeps 10000 --ladders 64 16
"""
import argparse
import json
import sys

import numpy as np

from . import analysis as A

NAMES = ("e", "|m|", "m2", "m4", "U_L")


def _series(sim, n_sweeps, n_metro, n_or, label="", chunk=1000):
    """Every sweep's observables, shape (n_sweeps, R_total, 5); the chain runs
    in chunks of ``chunk`` sweeps (one continuing chain) with a progress line
    on stderr after each."""
    import torch
    obs = torch.zeros((n_sweeps, sim.R_total, 5), dtype=torch.float64, device=sim.device)
    for t0 in range(0, n_sweeps, chunk):
        t1 = min(n_sweeps, t0 + chunk)
        sim.run(t1 - t0, n_metro, n_or, exchange_every=1, obs=obs[t0:t1])
        torch.cuda.synchronize()
        print(f"[precision] {label} {t1}/{n_sweeps} sweeps", file=sys.stderr, flush=True)
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
    o32 = _series(s32, n_sweeps, n_metro, n_or, "fp32")
    o64 = _series(s64, n_sweeps, n_metro, n_or, "fp64")
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


def _ladder_means(sim, n_ladders, n_sweeps, n_metro, n_or, discard, label=""):
    """Per ladder and beta position: long-run means of (E, e, |m|, m^2, m^4)
    after dropping the first ``discard`` fraction, shape (n_ladders, R, 5)."""
    o = _series(sim, n_sweeps, n_metro, n_or, f"{label} x {n_ladders} ladders")
    o = o[int(discard * n_sweeps):]
    return o.mean(axis=0).reshape(n_ladders, -1, 5)


def _mean_se(x):
    return float(x.mean()), float(x.std(ddof=1) / np.sqrt(len(x)))


def _binder_jk(m):
    """U_L (Eq. (5)) of the ensemble-mean m^2, m^4 at each beta and its
    leave-one-ladder-out jackknife error; m has shape (K, R, 5)."""
    K = m.shape[0]
    u = lambda a: 1.0 - a[..., 4] / (3.0 * a[..., 3] ** 2)
    full = u(m.mean(axis=0))
    loo = np.stack([u(np.delete(m, i, axis=0).mean(axis=0)) for i in range(K)])
    err = np.sqrt((K - 1) / K * ((loo - loo.mean(axis=0)) ** 2).sum(axis=0))
    return full, err


def compare_ladders(L, betas, n32=64, n64=16, n_sweeps=10000, n_metro=1, n_or=8, seeds=(3, 1003),
                    discard=0.2):
    """Ensemble form of the study: n32 float32 and n64 float64 independent
    ladders; per observable the difference of the ladder averages (mean over
    the betas) and per beta the difference of the ensemble means, each in
    units of the standard error from the spread of the ladders (U_L: the
    leave-one-ladder-out jackknife)."""
    from .sim import Sim

    if n32 < 2 or n64 < 2:
        raise ValueError("need at least two ladders per precision for a spread")
    R = len(betas)
    m = {}
    for prec, K, seed in (("fp32", n32, seeds[0]), ("fp64", n64, seeds[1])):
        s = Sim([L] * K, [list(map(float, betas))] * K, seed=seed, prec=prec)
        m[prec] = _ladder_means(s, K, n_sweeps, n_metro, n_or, discard, prec)
        s.close()
    a, b = m["fp32"], m["fp64"]
    ladder = {}
    for c, name in zip((1, 2, 3, 4), NAMES[:4]):
        (ma, ea), (mb, eb) = _mean_se(a[:, :, c].mean(axis=1)), _mean_se(b[:, :, c].mean(axis=1))
        err = float(np.hypot(ea, eb))
        ladder[name] = {"fp32": ma, "fp32_se": ea, "fp64": mb, "fp64_se": eb, "err": err,
                        "z": (ma - mb) / err}
    ua, uea = _binder_jk(a)
    ub, ueb = _binder_jk(b)
    per_beta, zs = [], []
    for k in range(R):
        row = {"beta": float(betas[k])}
        for c, name in zip((1, 2, 3, 4), NAMES[:4]):
            (ma, ea), (mb, eb) = _mean_se(a[:, k, c]), _mean_se(b[:, k, c])
            err = float(np.hypot(ea, eb))
            row[name] = {"fp32": ma, "fp64": mb, "err": err, "z": (ma - mb) / err}
            zs.append(row[name]["z"])
        err = float(np.hypot(uea[k], ueb[k]))
        row["U_L"] = {"fp32": float(ua[k]), "fp64": float(ub[k]), "err": err,
                      "z": float((ua[k] - ub[k]) / err)}
        zs.append(row["U_L"]["z"])
        per_beta.append(row)
    zs = np.array(zs)
    return {"L": L, "betas": [float(x) for x in betas], "n_sweeps": n_sweeps, "n_metro": n_metro,
            "n_or": n_or, "seeds": list(seeds), "discard": discard, "ladders": [n32, n64],
            "ladder_average": ladder,
            "max_abs_z": float(np.max(np.abs(zs))), "mean_z": float(np.mean(zs)),
            "rms_z": float(np.sqrt(np.mean(zs ** 2))), "n_compared": int(zs.size),
            "frac_within_2sigma": float(np.mean(np.abs(zs) <= 2.0)), "per_beta": per_beta}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--beta", type=float, nargs=2, default=[0.4530, 0.4554])
    ap.add_argument("--replicas", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=10000)
    ap.add_argument("--n-or", type=int, default=8)
    ap.add_argument("--seeds", type=int, nargs=2, default=[3, 1003])
    ap.add_argument("--ladders", type=int, nargs=2, metavar=("K32", "K64"),
                    help="ensemble form: K32 float32 and K64 float64 independent ladders")
    args = ap.parse_args(argv)
    betas = np.linspace(args.beta[0], args.beta[1], args.replicas)
    if args.ladders:
        res = compare_ladders(args.L, betas, n32=args.ladders[0], n64=args.ladders[1],
                              n_sweeps=args.sweeps, n_or=args.n_or, seeds=tuple(args.seeds))
    else:
        res = compare(args.L, betas, n_sweeps=args.sweeps, n_or=args.n_or, seeds=tuple(args.seeds))
    json.dump(res, sys.stdout)
    print()


if __name__ == "__main__":
    main()
