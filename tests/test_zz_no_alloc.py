"""The allocation-free sampled read-back xy_get_sites_noalloc, through the C
ABI, against xy_get_sites (the entry point it is a variant of): bit-identical
angles on two calls in a row, the second with a smaller input, FP32 and FP64;
sizes beyond the static scratch are rejected with an error."""
import ctypes

import numpy as np
import pytest

from paper_1211_0780_amd import _capi as C

pytestmark = pytest.mark.gpu


def _read(fn, sim, sites, lattice, beta_pos):
    idx = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.full(idx.size, np.nan)
    st = fn(sim._ctx, lattice, beta_pos, idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    C.check(st, sim._ctx)
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_read_back_equals_allocating_one(gpu, prec):
    from paper_1211_0780_amd.sim import Sim
    lib = C.lib()
    s = Sim([24, 10], [[0.44, 0.45, 0.46], [0.45]], seed=12, prec=prec)
    s.run(3, 1, 2, exchange_every=1)
    rng = np.random.default_rng(5)
    calls = [(0, 1, rng.integers(0, 24 ** 3, 9000)),           # first call: 9000 sites
             (1, 0, rng.integers(0, 10 ** 3, 37))]            # second call: fewer sites, other lattice
    for lattice, k, sites in calls:
        want = _read(lib.xy_get_sites, s, sites, lattice, k)
        got = _read(lib.xy_get_sites_noalloc, s, sites, lattice, k)
        assert np.array_equal(got, want), (lattice, k, sites.size)
        assert np.array_equal(got, s.get_angles(lattice, k)[sites])
    # the largest accepted size, then one past it
    big = rng.integers(0, 24 ** 3, C.XY_NOALLOC_MAX_SITES)
    assert np.array_equal(_read(lib.xy_get_sites_noalloc, s, big, 0, 2), _read(lib.xy_get_sites, s, big, 0, 2))
    with pytest.raises(C.XYError) as e:
        _read(lib.xy_get_sites_noalloc, s, np.zeros(C.XY_NOALLOC_MAX_SITES + 1, np.int64), 0, 0)
    assert e.value.status == C.XY_ERR_ARG
    # an empty request and an out-of-range site
    assert _read(lib.xy_get_sites_noalloc, s, np.zeros(0, np.int64), 0, 0).size == 0
    with pytest.raises(C.XYError):
        _read(lib.xy_get_sites_noalloc, s, np.array([24 ** 3]), 0, 0)
    s.close()
