"""Fit the float32 polynomial kernels used by the FP32 HIP path.

  atan(q)/pi  ~ q * A(q^2),   q in [0, 1]            (A: degree NA in q^2;
                                                      odd, so the same error on
                                                      [-1, 1], where the kernels
                                                      evaluate it)
  sin(2 pi r) ~ r * S(r^2),   cos(2 pi r) ~ C(r^2),   r in [-1/8, 1/8] turns

Coefficients come from a weighted least-squares fit on Chebyshev nodes refined
by a few Lawson (iteratively reweighted) passes toward the minimax solution,
then the float32 Horner evaluation is checked on a dense grid.  Run:
    python fit_polys.py
and paste the printed constants into xy_device.h (the kernels use the
degree-13 atan fit, NA = 7, and the degree-7 sine / degree-8 cosine fit
behind XY_POLY_SINCOS).
"""
import numpy as np


def lawson(f, basis, x, iters=60):
    w = np.ones_like(x)
    B = basis(x)
    for _ in range(iters):
        W = np.sqrt(w)[:, None]
        c, *_ = np.linalg.lstsq(B * W, f * W[:, 0], rcond=None)
        err = np.abs(B @ c - f)
        w = w * (err + 1e-300)
        w /= w.sum()
    return c


def horner32(c, s):
    acc = np.float32(c[-1]) * np.ones_like(s, dtype=np.float32)
    for ck in c[-2::-1]:
        acc = (acc * s + np.float32(ck)).astype(np.float32)
    return acc


def fit_atan(NA=7):
    q = np.cos(np.linspace(0, np.pi, 4000)) * 0.5 + 0.5
    f = np.arctan(q) / np.pi
    basis = lambda x: np.stack([x ** (2 * k + 1) for k in range(NA)], axis=1)
    # relative-ish weighting is not needed: the result feeds an absolute angle
    c = lawson(f, basis, q)
    qq = np.linspace(0, 1, 2_000_001).astype(np.float32)
    s = (qq * qq).astype(np.float32)
    approx = (qq * horner32(c, s)).astype(np.float32)
    err = np.abs(approx.astype(np.float64) - np.arctan(qq.astype(np.float64)) / np.pi)
    return c, err.max()


def fit_sincos(NS=4, NC=5):
    r = np.cos(np.linspace(0, np.pi, 4000)) / 8
    cs = lawson(np.sin(2 * np.pi * r), lambda x: np.stack([x ** (2 * k + 1) for k in range(NS)], 1), r)
    cc = lawson(np.cos(2 * np.pi * r), lambda x: np.stack([x ** (2 * k) for k in range(NC)], 1), r)
    rr = np.linspace(-0.125, 0.125, 2_000_001).astype(np.float32)
    s2 = (rr * rr).astype(np.float32)
    es = np.abs((rr * horner32(cs, s2)).astype(np.float64) - np.sin(2 * np.pi * rr.astype(np.float64))).max()
    ec = np.abs(horner32(cc, s2).astype(np.float64) - np.cos(2 * np.pi * rr.astype(np.float64))).max()
    return cs, cc, es, ec


if __name__ == "__main__":
    for NA in (6, 7, 8):
        c, e = fit_atan(NA)
        print(f"atan/pi degree {2 * NA - 1}: max abs err (turns) {e:.3e}")
        print("  ", ", ".join(f"{np.float32(v).item()!r}f" for v in c))
    for NS, NC in ((4, 4), (4, 5), (5, 5)):
        cs, cc, es, ec = fit_sincos(NS, NC)
        print(f"sin deg {2 * NS - 1} err {es:.3e}; cos deg {2 * NC - 2} err {ec:.3e}")
        print("  S:", ", ".join(f"{np.float32(v).item()!r}f" for v in cs))
        print("  C:", ", ".join(f"{np.float32(v).item()!r}f" for v in cc))
