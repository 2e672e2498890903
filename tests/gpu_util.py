"""Helpers shared by the GPU parity tests (comparison only, no method arithmetic)."""
import numpy as np

TWO_PI = 2 * np.pi


def circ(a, b):
    """Circular distance between angle arrays (radians)."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) % TWO_PI
    return np.minimum(d, TWO_PI - d)


def colour_mask(L, c):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return (((x + y + z) & 1) == c).ravel()


def field_numpy(theta, L):
    """Neighbour field h = sum of the six neighbouring unit vectors (numpy rolls)."""
    g = np.asarray(theta, dtype=np.float64).reshape(L, L, L)
    hx = sum(np.cos(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    hy = sum(np.sin(np.roll(g, s, axis=a)) for a in range(3) for s in (1, -1)).ravel()
    return hx, hy


def gpu_states(sim, lattice=0):
    return np.stack([sim.get_angles(lattice, k) for k in range(sim.R[lattice])])


def check_metro_half(start, got, ref, margin, L, colour, tol, band=1e-6):
    """One Metropolis half-sweep of one configuration: `got` (GPU) and `ref`
    (oracle) both from `start`; `margin` = oracle.metro_margin of the same
    half-sweep.  Every site of the colour agrees within `tol` rad, except
    decisions taken the other way, which must lie within `band` of the
    threshold (|u - exp(-beta dE)| < band).  Sites of the other colour are
    untouched.  Returns the number of such flipped decisions."""
    m = colour_mask(L, colour)
    assert np.array_equal(got[~m], start[~m]), "sites of the other colour changed"
    d = circ(got, ref)
    off = m & (d > tol)
    assert np.all(np.abs(margin[off]) < band), (np.flatnonzero(off)[:8], margin[off][:8], d[off][:8])
    return int(off.sum())


def or_bound(start, L, fp64=False):
    """Per-site bound of one over-relaxation update from `start`: the
    reflection angle's rounding error grows as 1/|h| (FP32: 16 * 2^-24 * 6 / |h|,
    at least 2e-5 rad; FP64: the same with 2^-53, at least 1e-12 rad)."""
    hx, hy = field_numpy(start, L)
    h = np.maximum(np.hypot(hx, hy), 1e-300)
    if fp64:
        return np.maximum(1e-12, 16 * 6 * 2.0 ** -53 / h)
    return np.maximum(2e-5, 16 * 2.0 ** -24 * 6 / h)


def check_or_substep(start, got, L, fp64=False):
    """One over-relaxation substep (colour 0, then colour 1) of one
    configuration against the oracle, colour by colour: colour 0 from
    `start`, colour 1 from `start` with the GPU's colour 0.  Returns the
    largest deviation in units of the per-site bound."""
    import oracle
    m0 = colour_mask(L, 0)
    worst = 0.0
    base = np.ascontiguousarray(start, dtype=np.float64)
    for colour, mask in ((0, m0), (1, ~m0)):
        ref = base.copy()
        oracle.or_half(ref, L, colour)
        r = circ(got, ref) / or_bound(base, L, fp64)
        assert np.all(r[mask] <= 1.0), (colour, np.flatnonzero(r[mask] > 1.0)[:8])
        worst = max(worst, float(r[mask].max()))
        base = np.where(m0, got, base) if colour == 0 else base
    return worst


# Measured on gfx950 over x = i / 2^24: the hardware sine and cosine of an
# angle in turns return unit vectors that are short by 3.23e-8 on average
# (the polynomial alternative: 5e-9), so every float32 bond term
# S_i . S_j = |S_i| |S_j| cos(theta_i - theta_j) is scaled by about
# 1 - 6.5e-8 and the float32 energy carries that relative bias.  Bound: twice
# the bias on |E|, plus the random rounding of N/2 float32 terms of size <= 6.
AMPLITUDE_DEFICIT = 3.3e-8


def e_tol_fp32(E_ref, N):
    return 2 * (2 * AMPLITUDE_DEFICIT) * abs(E_ref) + 4 * 6 * 2.0 ** -24 * np.sqrt(N)
