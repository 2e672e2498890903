"""CPU FP64 oracle of the 3D XY model hot path (arXiv:1211.0780, Sec. II).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  The C source
``xy_oracle.c`` holds the arithmetic; this module only loads it with ctypes
and marshals numpy arrays.  It shares no code with the HIP library.

Angles are float64 radians in natural site order i = x + L*(y + L*z), one
array of N = L**3 per configuration; a lattice's R configurations are stacked
by beta-position.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xy_oracle.c")
# XY_ORACLE_LIB points the loader at another build of the same source (used to
# check, on the CPU, that the pins reject deliberately broken oracles).
_LIB_PATH = os.environ.get("XY_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

PHASE_INIT, PHASE_METRO, PHASE_EXCH = 1, 2, 3


def build(force=False):
    """Compile the oracle with the host C compiler (plain -O2, no fast-math)."""
    if os.environ.get("XY_ORACLE_LIB"):
        return _LIB_PATH
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        c_int, c_u32, c_u64, c_dbl = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [c_u32]
        L.orc_uniform.restype = c_dbl
        L.orc_init.argtypes = [dp, c_int, c_int, c_int, c_u64]
        L.orc_init.restype = None
        L.orc_metro_half.argtypes = [dp, c_int, c_dbl, c_u64, c_u32, c_int, c_int, c_int, c_dbl, c_int]
        L.orc_metro_half.restype = ctypes.c_int64
        L.orc_metro_site.argtypes = [dp, c_int, c_dbl, c_u64, c_u32, c_int, c_int, c_int, c_dbl,
                                     ctypes.c_int64]
        L.orc_metro_site.restype = c_int
        L.orc_metro_margin.argtypes = [dp, c_int, c_dbl, c_u64, c_u32, c_int, c_int, c_int, c_dbl,
                                       c_int, dp]
        L.orc_metro_margin.restype = None
        L.orc_or_site.argtypes = [dp, c_int, ctypes.c_int64]
        L.orc_or_site.restype = None
        L.orc_or_half.argtypes = [dp, c_int, c_int]
        L.orc_or_half.restype = None
        L.orc_sweep.argtypes = [dp, c_int, c_int, dp, c_u64, c_u32, c_int, c_int, c_int, c_dbl, i64p]
        L.orc_sweep.restype = None
        L.orc_measure.argtypes = [dp, c_int, dp]
        L.orc_measure.restype = None
        L.orc_bond_sums.argtypes = [dp, c_int, dp]
        L.orc_bond_sums.restype = None
        L.orc_exchange.argtypes = [dp, dp, c_int, c_int, dp, c_u64, c_u32, c_int, i64p]
        L.orc_exchange.restype = c_int
        L.orc_run.argtypes = [dp, c_int, c_int, dp, c_u64, c_int, c_int, c_u32, c_u32, c_int,
                              c_int, c_int, c_dbl, c_int, dp, i64p, i64p]
        L.orc_run.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i64p(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _f64(theta):
    a = np.ascontiguousarray(theta, dtype=np.float64)
    return a


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[0], o[1], o[2], o[3]]


def uniform(word):
    return lib().orc_uniform(int(word) & 0xFFFFFFFF)


def init(L, R, seed, lat=0):
    """Random start of R configurations: theta = 2*pi*U(Philox INIT)."""
    th = np.empty((R, L ** 3), dtype=np.float64)
    lib().orc_init(_dp(th), L, R, lat, seed)
    return th


def metro_half(theta, L, beta, seed, t, lat, k, substep, colour, window=0.0):
    """In place on one configuration (float64 array of N).  Returns accepts.
    window = 0: uniform proposal; window w > 0: theta + w (U - 1/2)."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous and theta.size == L ** 3
    return lib().orc_metro_half(_dp(theta), L, float(beta), seed, t, lat, k, substep, float(window),
                                colour)


def metro_site(theta, L, beta, seed, t, lat, k, substep, i, window=0.0):
    """Metropolis update of site i alone (in place); returns 1 if accepted."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous and theta.size == L ** 3
    return lib().orc_metro_site(_dp(theta), L, float(beta), seed, t, lat, k, substep, float(window),
                                int(i))


def metro_margin(theta, L, beta, seed, t, lat, k, substep, colour, window=0.0):
    """U(b) - exp(-beta dE) of every site of one colour of a Metropolis
    half-sweep from ``theta`` (NaN at sites of the other colour); the move is
    taken where it is negative."""
    th = _f64(theta)
    assert th.size == L ** 3
    out = np.empty(L ** 3, dtype=np.float64)
    lib().orc_metro_margin(_dp(th), L, float(beta), seed, t, lat, k, substep, float(window),
                           colour, _dp(out))
    return out


def or_site(theta, L, i):
    """Over-relaxation of site i alone (in place)."""
    assert theta.dtype == np.float64 and theta.flags.c_contiguous and theta.size == L ** 3
    lib().orc_or_site(_dp(theta), L, int(i))


def or_half(theta, L, colour):
    assert theta.dtype == np.float64 and theta.flags.c_contiguous and theta.size == L ** 3
    lib().orc_or_half(_dp(theta), L, colour)


def sweep(theta, L, beta, seed, t, lat, n_metro, n_or, window=0.0):
    """In place on (R, N) configurations by beta-position.  Returns accepts per k."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    R = beta.size
    assert theta.dtype == np.float64 and theta.flags.c_contiguous and theta.size == R * L ** 3
    acc = np.zeros(R, dtype=np.int64)
    lib().orc_sweep(_dp(theta), L, R, _dp(beta), seed, t, lat, n_metro, n_or, float(window), _i64p(acc))
    return acc


def measure(theta, L):
    """(E, e, |m|, m^2, m^4) of one configuration."""
    th = _f64(theta)
    out = np.zeros(5)
    lib().orc_measure(_dp(th), L, _dp(out))
    return out


def bond_sums(theta, L):
    """(C_x, C_y, C_z, I_x, I_y, I_z) of one configuration (Eq. (6) inputs)."""
    th = _f64(theta)
    out = np.zeros(6)
    lib().orc_bond_sums(_dp(th), L, _dp(out))
    return out


def exchange(theta, E, L, beta, seed, tau, lat=0, n_acc=None):
    """In place on (R, N) configurations (or None) and energies E (R,)."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    R = beta.size
    assert E.dtype == np.float64 and E.flags.c_contiguous and E.size == R
    tp = None if theta is None else _dp(theta)
    return lib().orc_exchange(tp, _dp(E), L, R, _dp(beta), seed, tau, lat, _i64p(n_acc))


def run(L, beta, seed, n_sweeps, n_metro, n_or, exchange_every=1, lat=0, ordered=False,
        t0=0, tau0=0, window=0.0):
    """A whole run; returns (theta (R,N), obs (n_sweeps,R,5), metro accepts (R,),
    swap accepts (R,))."""
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    R = beta.size
    th = np.empty((R, L ** 3), dtype=np.float64)
    obs = np.zeros((n_sweeps, R, 5), dtype=np.float64)
    macc = np.zeros(R, dtype=np.int64)
    sacc = np.zeros(R, dtype=np.int64)
    lib().orc_run(_dp(th), L, R, _dp(beta), seed, lat, int(ordered), t0, tau0, n_sweeps,
                  n_metro, n_or, float(window), exchange_every, _dp(obs), _i64p(macc), _i64p(sacc))
    return th, obs, macc, sacc
