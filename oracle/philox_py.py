"""Philox4x32-10 in pure Python integers (test infrastructure only).

A second, independent rendering of the published Philox4x32-10 definition
(Salmon, Moraes, Dror, Shaw, SC'11), used to cross-check the C oracle and the
HIP device generator word for word.  Ten rounds; each round forms the exact
64-bit products M0*c0 and M1*c2 and permutes/xors their halves with the other
two counter words and the round key; the key is advanced by the Weyl
constants between rounds.
"""

MASK32 = 0xFFFFFFFF
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85

PHASE_INIT, PHASE_METRO, PHASE_EXCH = 1, 2, 3


def philox4x32_10(ctr, key):
    """Return the four 32-bit output words for counter ``ctr`` (4 words) and
    key ``key`` (2 words)."""
    c = [int(v) & MASK32 for v in ctr]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & MASK32
            k1 = (k1 + _W1) & MASK32
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 & MASK32, (p0 >> 32) ^ c[3] ^ k1, p0 & MASK32]
    return c


def key_of(seed):
    """Key words of a 64-bit seed: (low half, high half)."""
    return (seed & MASK32, (seed >> 32) & MASK32)


def counter(c0, c1, lat, pos, phase, substep):
    """Counter of one draw: (site or pair, sweep or exchange step,
    (lattice << 16) | beta-position, (phase << 24) | substep)."""
    return (c0 & MASK32, c1 & MASK32, ((lat << 16) | pos) & MASK32,
            ((phase << 24) | substep) & MASK32)


def metro_words(i, L, t, lat, pos, substep, key):
    """The two words (proposal, acceptance) that site i = x + L (y + L z)
    draws in a Metropolis substep: the same-colour sites (x, y, 2m) and
    (x xor 1, y, 2m + 1) share the block whose first counter word is the
    even-plane site's index; the even-plane site takes words 0, 1 and the
    odd-plane site words 2, 3."""
    x, y, z = i % L, (i // L) % L, i // (L * L)
    i0 = (x ^ 1) + L * (y + L * (z - 1)) if z & 1 else i
    r = philox4x32_10(counter(i0, t, lat, pos, PHASE_METRO, substep), key)
    w = 2 * (z & 1)
    return r[w], r[w + 1]


def uniform(word):
    """U(r) = (r >> 8) * 2^-24, exactly representable in float32 and float64."""
    return (word >> 8) * (1.0 / 16777216.0)
