"""Reduced-precision storage as the oracle models it (test infrastructure).

bfloat16 keeps the top 16 bits of an IEEE binary32 value; rounding to it is
to nearest with ties to even.  A complex value is rounded part by part.  The
oracle feeds operators built from such rounded maps to the same FP64
arithmetic as everywhere else, so a GPU run with bfloat16 map storage can be
compared with the operator it actually applies.
"""
from __future__ import annotations

import numpy as np

from .sense import whiten_maps


def bf16_round_real(x) -> np.ndarray:
    """Values of float32(x) rounded to bfloat16 (nearest, ties to even), as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(nan, ((u >> 16) | 0x40) << 16, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_round(z) -> np.ndarray:
    """Complex array rounded part by part through complex64 to bfloat16."""
    z = np.asarray(z, np.complex64)
    return bf16_round_real(z.real) + 1j * bf16_round_real(z.imag)


def bf16_whitened_maps(maps, psi) -> np.ndarray:
    """Whitened maps S_w = L^-1 S of complex64 input maps, rounded to complex64
    and then to bfloat16: the maps of an operator stored in bfloat16 (its
    noise covariance is then the identity)."""
    w = whiten_maps(np.asarray(maps, np.complex64), psi)
    return bf16_round(w.astype(np.complex64))
