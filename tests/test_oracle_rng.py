"""Pins of the oracle's random-number stream (Philox4x32-10 and the uniform map).

The external pin is rocRAND's installed Philox4x32-10 block function, compiled
here as a host program; the Python big-int rendering is a second independent
implementation.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle.philox_py as P

HERE = os.path.dirname(os.path.abspath(__file__))


def _edge_and_random_cases(n, seed=12345):
    rng = np.random.default_rng(seed)
    cases = [
        ((0, 0), (0, 0, 0, 0)),
        ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFFF,) * 4),
        ((1, 0), (0, 0, 0, 0)),
        ((0, 1), (0, 0, 0, 0)),
        ((0, 0), (1, 0, 0, 0)),
        ((0, 0), (0, 0, 0, 1)),
    ]
    for _ in range(n):
        k = tuple(int(v) for v in rng.integers(0, 2 ** 32, 2, dtype=np.uint64))
        c = tuple(int(v) for v in rng.integers(0, 2 ** 32, 4, dtype=np.uint64))
        cases.append((k, c))
    return cases


@pytest.fixture(scope="module")
def rocrand_dump(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host helper")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_dump")
    subprocess.check_call([hipcc, "-O1", os.path.join(HERE, "helpers", "rocrand_philox_dump.cpp"),
                           "-o", exe])
    return exe


def test_oracle_matches_rocrand(orc, rocrand_dump):
    cases = _edge_and_random_cases(3000)
    text = "".join(f"{k[0]} {k[1]} {c[0]} {c[1]} {c[2]} {c[3]}\n" for k, c in cases)
    out = subprocess.run([rocrand_dump], input=text, capture_output=True, text=True, check=True)
    ref = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for (k, c), r in zip(cases, ref):
        assert orc.philox(c, k) == r, (k, c)


def test_oracle_matches_python_bigint(orc):
    for k, c in _edge_and_random_cases(2000, seed=7):
        assert orc.philox(c, k) == P.philox4x32_10(c, k)


def test_philox_avalanche(orc):
    """Flipping one counter bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(200):
        k = [int(v) for v in rng.integers(0, 2 ** 32, 2, dtype=np.uint64)]
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4, dtype=np.uint64)]
        w = int(rng.integers(0, 4))
        b = int(rng.integers(0, 32))
        c2 = list(c)
        c2[w] ^= 1 << b
        a, bb = orc.philox(c, k), orc.philox(c2, k)
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, bb)))
    assert 60 < np.mean(flips) < 68


def test_uniform_map(orc):
    assert orc.uniform(0) == 0.0
    assert orc.uniform(0xFF) == 0.0
    assert orc.uniform(0x100) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    # exactly representable in float32 as well
    for w in (0x12345678, 0xDEADBEEF, 0x80000000):
        u = orc.uniform(w)
        assert float(np.float32(u)) == u
        assert u == P.uniform(w)


def test_uniform_moments(orc):
    key = P.key_of(99)
    us = np.array([orc.uniform(orc.philox((i, 0, 0, 0), key)[0]) for i in range(20000)])
    assert abs(us.mean() - 0.5) < 4 * np.sqrt(1 / 12 / us.size)
    assert abs((us ** 2).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / us.size)


def test_init_is_two_pi_uniform(orc):
    L, R, seed, lat = 4, 3, 0x1234_5678_9ABC_DEF0, 2
    th = orc.init(L, R, seed, lat)
    key = P.key_of(seed)
    for k in range(R):
        for i in (0, 1, 17, L ** 3 - 1):
            r = P.philox4x32_10(P.counter(i, 0, lat, k, P.PHASE_INIT, 0), key)
            assert th[k, i] == 2 * np.pi * P.uniform(r[0])
    assert th.min() >= 0.0 and th.max() < 2 * np.pi


@pytest.mark.parametrize("L", [4, 6])
def test_metropolis_words_are_distinct_and_paired(L):
    """Every site of a substep reads its own pair of words, and a block serves
    exactly two sites of one colour on planes 2m and 2m + 1: the even-plane
    site (whose index is the block's counter word) and its x-neighbour's
    same-colour partner one plane up."""
    key = P.key_of(5)
    seen, blocks = {}, {}
    for i in range(L ** 3):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        words = P.metro_words(i, L, 3, 0, 1, 0, key)
        assert words not in seen, (i, seen.get(words))
        seen[words] = i
        i0 = (x ^ 1) + L * (y + L * (z - 1)) if z & 1 else i
        full = P.philox4x32_10(P.counter(i0, 3, 0, 1, P.PHASE_METRO, 0), key)
        assert words == tuple(full[2 * (z & 1): 2 * (z & 1) + 2])
        blocks.setdefault(i0, []).append((x + y + z) & 1)
    assert len(blocks) == L ** 3 // 2
    assert all(len(c) == 2 and c[0] == c[1] for c in blocks.values())
