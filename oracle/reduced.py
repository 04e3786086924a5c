"""Reduced-resolution noise grid (Sec. 5, Discussion: noise maps follow the
smooth coil geometry, so the variance can be estimated on a coarser grid and
interpolated back to the native one).  Test infrastructure: a plain FP64
statement of the coarse problem and of the interpolation.

Reading of the paper (it gives no construction): the coarse problem of
factor f is the same acquisition restricted to the central (ny/f) x (nx/f)
block of k-space, reconstructed on an (ny/f) x (nx/f) grid.  With the
centred orthonormal DFT, coarse pixel m sits at native pixel f m (both grids
keep the centre pixel N/2), so the coarse maps are the native maps sampled
at every f-th pixel and the coarse mask is the central block of the native
mask; a non-Cartesian sample w (rad per native pixel) enters the coarse
problem as f w when |w_y|, |w_x| < pi / f.  White k-space noise of unit
variance keeps unit variance, and an orthonormal transform keeps the pixel
variance level, so the coarse variance map estimates the native one at the
coarse pixels with no rescaling.  Back to the native grid by periodic
bilinear interpolation between the coarse pixels.
"""
from __future__ import annotations

import numpy as np


def coarse_maps(maps, f: int) -> np.ndarray:
    """Native maps [nc][ny][nx] sampled at native pixels (f my, f mx)."""
    maps = np.asarray(maps)
    return maps[:, ::f, ::f].copy()


def coarse_mask(mask, f: int) -> np.ndarray:
    """Central block of a centred-order mask: [ny] -> [ny/f], [ny][nx] -> [ny/f][nx/f]."""
    mask = np.asarray(mask)
    out = mask
    for ax in range(mask.ndim):
        n = mask.shape[ax]
        lo = (n - n // f) // 2
        out = np.take(out, np.arange(lo, lo + n // f), axis=ax)
    return out.copy()


def coarse_traj(traj, f: int) -> np.ndarray:
    """Samples inside the coarse band, in rad per coarse pixel (order kept)."""
    traj = np.asarray(traj, np.float64)
    lim = np.pi / f
    keep = np.all((traj >= -lim) & (traj < lim), axis=1)
    return traj[keep] * f


def upsample_bilinear(coarse, f: int) -> np.ndarray:
    """Native map [f cy][f cx] from a coarse one: native pixel (y, x) lies at
    coarse coordinate (y / f, x / f); periodic bilinear weights."""
    coarse = np.asarray(coarse, np.float64)
    cy, cx = coarse.shape
    ny, nx = f * cy, f * cx
    out = np.empty((ny, nx))
    for y in range(ny):
        y0, ty = divmod(y, f)
        wy = ty / f
        for x in range(nx):
            x0, tx = divmod(x, f)
            wx = tx / f
            a = coarse[y0, x0]
            b = coarse[y0, (x0 + 1) % cx]
            c = coarse[(y0 + 1) % cy, x0]
            d = coarse[(y0 + 1) % cy, (x0 + 1) % cx]
            out[y, x] = (1 - wy) * ((1 - wx) * a + wx * b) + wy * ((1 - wx) * c + wx * d)
    return out
