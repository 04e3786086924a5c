"""Counter-based random numbers for probes and PMR noise (oracle side).

The paper draws random-phase probes v_k = exp(j theta_k), theta ~ U[0, 2 pi]
(Sec. 2.2, Eq. (20); App. A, Algorithm 1, step (1)).  To compare the GPU
path with this oracle on *identical* probes both sides implement the same
counter-based generator from its published definition: Philox4x32-10
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11).  Its round function: two multiply-hi/lo products of counter words 0
and 2 with the round multipliers, XOR of the high halves with the other
counter words and the key, a fixed word permutation, and a Weyl-sequence key
bump between rounds.  The 64-bit variant (Philox4x64-10) has the same
structure with 64-bit constants; numpy ships it as a library bit generator,
which pins this implementation's round structure (tests/test_oracle_philox.py).

Counter layout (a reading the paper leaves open; it only fixes the
distribution): key = (seed mod 2^32, seed >> 32); counter =
(element index, draw index mod 2^32, draw index >> 32, stream), where the
draw index is the probe (or replica) number and ``stream`` separates uses:
"""
from __future__ import annotations

import numpy as np

STREAM_PROBE = 0      # image-domain probes v^(i)
STREAM_PMR = 1        # k-space noise replicas
STREAM_JVP = 2        # k-space probes for the CS Jacobian
STREAM_POWER = 3      # power-method start vector

# Philox4x32 constants (Salmon et al., SC'11)
M32 = (0xD2511F53, 0xCD9E8D57)
W32 = (0x9E3779B9, 0xBB67AE85)
# Philox4x64 constants (same paper)
M64 = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
W64 = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)


def philox_scalar(ctr, key, bits=32, rounds=10):
    """Reference Philox4xW-R on Python integers (one block).

    ``ctr`` is 4 words, ``key`` 2 words, each < 2^bits.  Returns 4 words.
    """
    mask = (1 << bits) - 1
    M = M32 if bits == 32 else M64
    W = W32 if bits == 32 else W64
    c0, c1, c2, c3 = (int(v) & mask for v in ctr)
    k0, k1 = (int(v) & mask for v in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W[0]) & mask
            k1 = (k1 + W[1]) & mask
        p0 = M[0] * c0
        p1 = M[1] * c2
        hi0, lo0 = p0 >> bits, p0 & mask
        hi1, lo1 = p1 >> bits, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over numpy uint32 arrays (broadcasting)."""
    m32 = np.uint64(0xFFFFFFFF)
    c = [np.asarray(v, np.uint64) & m32 for v in (c0, c1, c2, c3)]
    c0, c1, c2, c3 = np.broadcast_arrays(*c)
    c0, c1, c2, c3 = (v.copy() for v in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    A, B = np.uint64(M32[0]), np.uint64(M32[1])
    sh = np.uint64(32)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W32[0]) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + W32[1]) & 0xFFFFFFFF)
        p0 = A * c0          # < 2^64: exact in uint64
        p1 = B * c2
        hi0, lo0 = p0 >> sh, p0 & m32
        hi1, lo1 = p1 >> sh, p1 & m32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def draw_words(seed: int, draw: int, nelem: int, stream: int):
    """Philox words for elements 0..nelem-1 of draw ``draw`` on ``stream``."""
    k = np.arange(nelem, dtype=np.uint64)
    d = int(draw)
    return philox4x32(k, d & 0xFFFFFFFF, (d >> 32) & 0xFFFFFFFF, stream,
                      seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def phase_fraction(w0):
    """24-bit phase fraction f = (w0 >> 8) / 2^24 in [0, 1), exact in float32."""
    return (np.asarray(w0, np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def probe(seed: int, draw: int, nelem: int, dist: str = "phase", stream: int = STREAM_PROBE):
    """One probe vector, complex128 [nelem].

    dist:
      "phase"      random phase exp(j 2 pi f)            (Sec. 2.2, Eq. (20))
      "qpsk"       exp(j pi/2 q), q = top 2 bits          (discrete random phase)
      "rademacher" +-1 from the top bit                   (Sec. 2.2, Eq. (19))
      "gaussian"   CN(0, 1) by Box-Muller (1958)           (Sec. 2.2, Eq. (18))
    All satisfy E[v] = 0, E[v v^H] = I (Sec. 2.2, Eq. (15)).
    """
    w0, w1, _, _ = draw_words(seed, draw, nelem, stream)
    if dist == "phase":
        f = phase_fraction(w0)
        return np.exp(2j * np.pi * f)
    if dist == "qpsk":
        q = (w0 >> np.uint32(30)).astype(np.int64)
        return (1j) ** q
    if dist == "rademacher":
        b = (w0 >> np.uint32(31)).astype(np.float64)
        return (1.0 - 2.0 * b).astype(np.complex128)
    if dist == "gaussian":
        u1 = ((w0 >> np.uint32(8)).astype(np.float64) + 1.0) * 2.0 ** -24   # (0, 1]
        u2 = phase_fraction(w1)
        r = np.sqrt(-np.log(u1))            # |z|^2 ~ Exp(1): E|z|^2 = 1
        return r * np.exp(2j * np.pi * u2)
    raise ValueError(dist)


DISTS = {"phase": 0, "qpsk": 1, "rademacher": 2, "gaussian": 3}
