"""Orthonormal periodised Daubechies wavelet transform, FP64 (oracle side).

The CS workload regularises with an L1 penalty on a 4-level db4 wavelet
transform (the paper's CS experiment used TV, Sec. 3.2.3; the wavelet
penalty is the reading taken for this workload).  No wavelet library is
available, so the db4 scaling filter is derived here by spectral
factorisation of the Daubechies polynomial (Daubechies, "Ten Lectures on
Wavelets", ch. 6):

  |m0(w)|^2 = cos^{2p}(w/2) P(sin^2(w/2)),  P(y) = sum_{k<p} C(p-1+k, k) y^k,

with p = 4 vanishing moments.  Each root y_r of P gives the pair of z-roots
of z + 1/z = 2 - 4 y_r; the one inside the unit circle is kept (minimum
phase), and h = sqrt(2) normalised coefficients of (1 + z^-1)^p prod (1 - z_r z^-1).
The high-pass filter is g[k] = (-1)^k h[L-1-k].

Periodised analysis along one axis of length n (even):
  a[i] = sum_k h[k] x[(2i + k) mod n],   d[i] = sum_k g[k] x[(2i + k) mod n],
stored as [a | d].  The 2-D level transforms rows, then columns, of the
current low-pass block; J levels recurse on the top-left block.
"""
from __future__ import annotations

from math import comb

import numpy as np


def daubechies_scaling(p: int = 4) -> np.ndarray:
    """Minimum-phase Daubechies scaling filter with p vanishing moments (2p taps)."""
    P = [comb(p - 1 + k, k) for k in range(p)]            # ascending powers of y
    yroots = np.roots(P[::-1])
    zr = []
    for y in yroots:
        r = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        zr.append(r[np.argmin(np.abs(r))])
    q = np.real(np.poly(zr))                              # prod (z - z_r), z-polynomial
    b = np.array([comb(p, k) for k in range(p + 1)], np.float64)   # (1 + z)^p
    h = np.convolve(b, q)
    h = h / h.sum() * np.sqrt(2.0)
    # order as coefficients of z^-k with the largest tap early (min phase)
    if abs(h[0]) < abs(h[-1]):
        h = h[::-1]
    return h


def wavelet_filter(p: int = 4):
    h = daubechies_scaling(p)
    L = h.size
    g = np.array([(-1) ** k * h[L - 1 - k] for k in range(L)])
    return h, g


def _analysis_axis(x, h, g, axis):
    x = np.moveaxis(x, axis, -1)
    n = x.shape[-1]
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(h.size)[None, :]) % n
    seg = x[..., idx]                                      # [..., n/2, L]
    a = seg @ h
    d = seg @ g
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def _synthesis_axis(c, h, g, axis):
    c = np.moveaxis(c, axis, -1)
    n = c.shape[-1]
    a, d = c[..., : n // 2], c[..., n // 2:]
    out = np.zeros(c.shape, np.result_type(c, np.float64))
    for k in range(h.size):
        pos = (2 * np.arange(n // 2) + k) % n
        np.add.at(out, (..., pos), a * h[k] + d * g[k])
    return np.moveaxis(out, -1, axis)


def wavedec2(x, levels: int = 4, p: int = 4):
    """J-level 2-D analysis; returns coefficients in one array of x's shape."""
    h, g = wavelet_filter(p)
    c = np.array(x, dtype=np.result_type(x, np.float64), copy=True)
    ny, nx = c.shape[-2:]
    for _ in range(levels):
        blk = c[..., :ny, :nx]
        blk = _analysis_axis(blk, h, g, -1)
        blk = _analysis_axis(blk, h, g, -2)
        c[..., :ny, :nx] = blk
        ny //= 2
        nx //= 2
    return c


def waverec2(c, levels: int = 4, p: int = 4):
    """Inverse of wavedec2 (its adjoint: the transform is orthonormal)."""
    h, g = wavelet_filter(p)
    x = np.array(c, dtype=np.result_type(c, np.float64), copy=True)
    ny, nx = x.shape[-2:]
    sizes = []
    for _ in range(levels):
        sizes.append((ny, nx))
        ny //= 2
        nx //= 2
    for ny, nx in reversed(sizes):
        blk = x[..., :ny, :nx]
        blk = _synthesis_axis(blk, h, g, -2)
        blk = _synthesis_axis(blk, h, g, -1)
        x[..., :ny, :nx] = blk
    return x


def detail_mask(shape, levels: int = 4) -> np.ndarray:
    """True on detail coefficients (everything but the coarsest low-pass block)."""
    m = np.ones(shape, bool)
    m[: shape[0] >> levels, : shape[1] >> levels] = False
    return m
