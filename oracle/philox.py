"""Philox4x64-10 counter-based random numbers (oracle side).

Written from the published definition of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two
64x64->128-bit multiplications with the multipliers M0, M1, the key bumped by
the Weyl constants W0, W1 between rounds.  The paper itself only has a seeds
file (section "Input files"); the addressing below is a reading of our own:

    key     = (chain seed, 0)
    counter = (stream tag, sweep, (tau << 1) | direction, site)
    u       = (word0 >> 11) * 2**-53            in [0, 1)

so that every draw is addressed by where it is used and batching or resuming
never changes a chain's random numbers.

Pinned in the tests against numpy.random.Philox (an independent
implementation of the same generator).
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
_MASK64 = (1 << 64) - 1

TAG_INIT = 0
TAG_FLIP = 1
TAG_GAUSS = 2
TAG_LANGEVIN = 3
DIR_UP = 0
DIR_DOWN = 1


def philox4x64_10(counter, key):
    """One Philox4x64-10 block with Python integers: returns four 64-bit words."""
    x0, x1, x2, x3 = (int(c) & _MASK64 for c in counter)
    k0, k1 = (int(k) & _MASK64 for k in key)
    for _ in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> 64, p0 & _MASK64
        hi1, lo1 = p1 >> 64, p1 & _MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + W0) & _MASK64
        k1 = (k1 + W1) & _MASK64
    return x0, x1, x2, x3


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: int, b: np.ndarray):
    """Full 64x64 -> 128-bit product of the constant a with each entry of b,
    from four 32x32-bit partial products (each exact in uint64)."""
    a_lo = np.uint64(a & 0xFFFFFFFF)
    a_hi = np.uint64(a >> 32)
    b_lo = b & _M32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | (mid << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10_vec(c0, c1, c2, c3, key):
    """Vectorised Philox4x64-10 over arrays of counters (uint64 arrays that
    broadcast together); returns four uint64 arrays."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3)))
        x0, x1, x2, x3 = (x.copy() for x in (x0, x1, x2, x3))
        k0 = int(key[0]) & _MASK64
        k1 = int(key[1]) & _MASK64
        for _ in range(10):
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
            k0 = (k0 + W0) & _MASK64
            k1 = (k1 + W1) & _MASK64
    return x0, x1, x2, x3


def to_unit(word) -> np.ndarray:
    """Top 53 bits of a 64-bit word as a double in [0, 1)."""
    return (np.asarray(word, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def slot(tau: int, direction: int) -> int:
    return (int(tau) << 1) | int(direction)


def uniforms(seed: int, tag: int, sweep: int, tau: int, direction: int, n: int, word: int = 0):
    """u for sites 0..n-1 at one (tag, sweep, tau, direction)."""
    w = philox4x64_10_vec(np.uint64(tag), np.uint64(sweep), np.uint64(slot(tau, direction)),
                          np.arange(n, dtype=np.uint64), (seed, 0))
    return to_unit(w[word])


def normals(seed: int, tag: int, sweep: int, tau: int, direction: int, n: int):
    """Standard normals by Box-Muller on (1 - u0, u1), cosine branch."""
    w = philox4x64_10_vec(np.uint64(tag), np.uint64(sweep), np.uint64(slot(tau, direction)),
                          np.arange(n, dtype=np.uint64), (seed, 0))
    u0 = to_unit(w[0])
    u1 = to_unit(w[1])
    return np.sqrt(-2.0 * np.log1p(-u0)) * np.cos(2.0 * np.pi * u1)
