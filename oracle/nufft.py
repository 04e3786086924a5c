"""Non-Cartesian SENSE operators, FP64 (oracle side).

The spiral experiments encode with a NUFFT and use a Toeplitz embedding for
the normal operator (Sec. 3.2.2; Sec. 3.3).  The paper gives neither the
NUDFT sign / scale nor the embedding; the readings here:

* Direct NUDFT (the operator the NUFFT approximates):
      (A u)_m = N_x^-1/2 sum_r u_r exp(-i w_m . r),
  with r the centred integer image coordinates (y - ny/2, x - nx/2) and
  w_m = (w_y, w_x) in radians, |w| < pi.  On grid-aligned trajectories
  (w = 2 pi k / n) this is exactly the centred orthonormal DFT used for the
  Cartesian path.
* Normal operator of one coil: (A^H A u)_r = sum_r' psf(r - r') u_r' with
      psf(d) = N_x^-1 sum_m exp(i w_m . d),   d in [-(n-1), n-1]^2,
  a Hermitian-symmetric kernel.  Embedded circulantly in a 2ny x 2nx grid
  (k[d mod 2n] = psf(d), zero at the index n), linear convolution becomes
  a 2n-point cyclic one: A^H A u = crop(IDFT(K^ . DFT(pad(u)))) with
  K^ = DFT(k) real.  This Toeplitz form equals the exact NUDFT normal
  operator up to rounding (pinned in tests/test_oracle_nufft.py).

Multi-coil whitened operators apply the same per coil with S_w,c = L^-1 S_c
(Sec. 2.1, Eq. (3)).  Everything is plain numpy; the exponentials are
evaluated separably, exp(-i w . r) = exp(-i w_y r_y) exp(-i w_x r_x), with
chunking over samples to bound memory.
"""
from __future__ import annotations

import numpy as np

from .sense import whiten_maps

_CHUNK = 8192


def centred(n: int) -> np.ndarray:
    return np.arange(n) - n // 2


def nudft_forward(u: np.ndarray, traj: np.ndarray) -> np.ndarray:
    """(A u)_m for one image u [ny][nx]; traj float [M][2] = (w_y, w_x)."""
    ny, nx = u.shape
    ry, rx = centred(ny), centred(nx)
    out = np.empty(traj.shape[0], np.complex128)
    for s in range(0, traj.shape[0], _CHUNK):
        w = traj[s:s + _CHUNK]
        Ey = np.exp(-1j * np.outer(w[:, 0], ry))          # [m][ny]
        Ex = np.exp(-1j * np.outer(w[:, 1], rx))          # [m][nx]
        out[s:s + _CHUNK] = np.sum((Ey @ u) * Ex, axis=1)
    return out / np.sqrt(ny * nx)


def nudft_adjoint(k: np.ndarray, traj: np.ndarray, shape) -> np.ndarray:
    """(A^H k)_r = N_x^-1/2 sum_m k_m exp(+i w_m . r), image [ny][nx]."""
    ny, nx = shape
    ry, rx = centred(ny), centred(nx)
    out = np.zeros((ny, nx), np.complex128)
    for s in range(0, traj.shape[0], _CHUNK):
        w = traj[s:s + _CHUNK]
        Ey = np.exp(1j * np.outer(w[:, 0], ry))
        Ex = np.exp(1j * np.outer(w[:, 1], rx))
        out += (Ey * k[s:s + _CHUNK, None]).T @ Ex
    return out / np.sqrt(ny * nx)


def psf(traj: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """psf(d) for d_y in [-(ny-1), ny-1], d_x in [-(nx-1), nx-1]; [2ny-1][2nx-1]."""
    dy = np.arange(-(ny - 1), ny)
    dx = np.arange(-(nx - 1), nx)
    out = np.zeros((dy.size, dx.size), np.complex128)
    for s in range(0, traj.shape[0], _CHUNK):
        w = traj[s:s + _CHUNK]
        Fy = np.exp(1j * np.outer(w[:, 0], dy))
        Fx = np.exp(1j * np.outer(w[:, 1], dx))
        out += Fy.T @ Fx
    return out / (ny * nx)


def toeplitz_kernel(traj: np.ndarray, ny: int, nx: int) -> np.ndarray:
    """K^ = DFT_{2ny x 2nx} of the circulant embedding of psf; float64 (real)."""
    p = psf(traj, ny, nx)
    k = np.zeros((2 * ny, 2 * nx), np.complex128)
    dy = np.arange(-(ny - 1), ny) % (2 * ny)
    dx = np.arange(-(nx - 1), nx) % (2 * nx)
    k[np.ix_(dy, dx)] = p
    kh = np.fft.fft2(k)
    assert np.abs(kh.imag).max() <= 1e-9 * np.abs(kh).max(), "Toeplitz kernel is not real"
    return kh.real


class NonCartOp:
    """Whitened non-Cartesian SENSE operator.

    ``normal`` uses the Toeplitz embedding, which equals the NUDFT's A^H A
    exactly, or, with ``normal_mode="gridding"``, the normal operator of the
    gridding NUFFT itself, sum_c S_c^H A_grid^H A_grid S_c (its plain
    definition: forward, then adjoint, per coil).  ``forward`` / ``adjoint``
    (the data path: reconstruction of k-space data and PMR replicas) are the
    direct NUDFT, or the Kaiser-Bessel gridding NUFFT of oracle/kbnufft.py when
    ``kb = (sigma, W)`` is given.
    """

    def __init__(self, maps, psi, traj, kb=None, normal_mode="toeplitz"):
        if normal_mode not in ("toeplitz", "gridding") or (normal_mode == "gridding" and kb is None):
            raise ValueError("normal_mode is 'toeplitz', or 'gridding' with kb = (sigma, W)")
        self.normal_mode = normal_mode
        self.Sw = whiten_maps(maps, psi)
        self.nc, self.ny, self.nx = self.Sw.shape
        self.traj = np.asarray(traj, np.float64)
        self.M = self.traj.shape[0]
        self.Kh = toeplitz_kernel(self.traj, self.ny, self.nx)
        self.kb = None
        if kb is not None:
            from .kbnufft import KBGridding
            self.kb = KBGridding(self.traj, self.ny, self.nx, *kb)

    def forward(self, x):
        """A x -> [nc][M]."""
        if self.kb is not None:
            return np.stack([self.kb.forward(self.Sw[c] * x) for c in range(self.nc)])
        return np.stack([nudft_forward(self.Sw[c] * x, self.traj) for c in range(self.nc)])

    def adjoint(self, y):
        """A^H y -> image."""
        if self.kb is not None:
            return sum(np.conj(self.Sw[c]) * self.kb.adjoint(y[c]) for c in range(self.nc))
        return sum(np.conj(self.Sw[c]) * nudft_adjoint(y[c], self.traj, (self.ny, self.nx))
                   for c in range(self.nc))

    def conv(self, u):
        """Per-coil normal operator (psf convolution) via the 2n embedding."""
        ny, nx = self.ny, self.nx
        pad = np.zeros((2 * ny, 2 * nx), np.complex128)
        pad[:ny, :nx] = u
        return np.fft.ifft2(self.Kh * np.fft.fft2(pad))[:ny, :nx]

    def normal(self, x):
        """M x = sum_c conj(S_c) psf * (S_c x) (Toeplitz), or
        sum_c conj(S_c) A_grid^H A_grid (S_c x) (gridding)."""
        if self.normal_mode == "gridding":
            return self.normal_gridding(x)
        return sum(np.conj(self.Sw[c]) * self.conv(self.Sw[c] * x) for c in range(self.nc))

    def normal_gridding(self, x):
        """M_grid x = sum_c conj(S_c) A_grid^H A_grid (S_c x), with the gridding NUFFT."""
        return sum(np.conj(self.Sw[c]) * self.kb.adjoint(self.kb.forward(self.Sw[c] * x))
                   for c in range(self.nc))

    def normal_nudft(self, x):
        """M x through the NUDFT forward and adjoint (slow; for checks)."""
        return self.adjoint(self.forward(x))

    def dense_normal(self):
        n = self.ny * self.nx
        Md = np.empty((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1
            Md[:, j] = self.normal(e.reshape(self.ny, self.nx)).ravel()
        return Md
