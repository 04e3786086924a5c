"""Kaiser-Bessel gridding NUFFT, FP64 (oracle side; test infrastructure only).

The spiral experiments reconstruct with a gridding NUFFT (Sec. 3.2.2 and
Sec. 3.3: SigPy's Kaiser-Bessel NUFFT, width 4, with a Toeplitz normal
operator).  The paper fixes neither the oversampling nor the kernel shape
parameter; the readings here:

* grid G = sigma N per axis (sigma N an integer), image zero-padded with the
  centred coordinate r at grid index r mod G, plain DFT on the grid
  (Y_k = sum_r y_r exp(-2 pi i k r / G));
* kernel phi(u) = I0(beta sqrt(1 - (2u/W)^2)) for |u| <= W/2 (u in grid
  cells), beta = pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8) (Beatty, Nishimura
  and Pauly, IEEE TMI 2005);
* a sample at w (rad) sits at kappa = w G / (2 pi) grid cells; its W taps per
  axis are k = floor(kappa) - W/2 + 1 + t, t = 0..W-1 (W even), indices mod G;
* de-apodisation by the kernel's continuous Fourier transform (Jackson et
  al., IEEE TMI 1991) at nu = r / G:
      Phi(nu) = W sinh(sqrt(beta^2 - (pi W nu)^2)) / sqrt(beta^2 - (pi W nu)^2)
  (the sin form when the root is imaginary);
* scale N_x^-1/2 so that the result approximates the direct NUDFT
  (A u)_m = N_x^-1/2 sum_r u_r exp(-i w_m . r) of oracle/nufft.py.

The adjoint is the exact adjoint of this linear map: spread with the same
weights, inverse (unnormalised, exp(+2 pi i k r / G)) DFT, crop, the same
de-apodisation and scale.  Separable in y and x.  I0 by its power series.
"""
from __future__ import annotations

import math

import numpy as np


def i0(x):
    """Modified Bessel function of the first kind, order 0, by its power series
    sum_k ((x/2)^2)^k / (k!)^2 (terms until they drop below 1e-17 of the sum)."""
    x = np.asarray(x, np.float64)
    q = (x / 2.0) ** 2
    term = np.ones_like(q)
    s = np.ones_like(q)
    k = 1
    while True:
        term = term * q / (k * k)
        s = s + term
        if np.all(term <= 1e-17 * s):
            break
        k += 1
    return s


def kb_beta(sigma: float, W: int) -> float:
    return math.pi * math.sqrt((W / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb_kernel(u, W: int, beta: float):
    u = np.asarray(u, np.float64)
    a = 1.0 - (2.0 * u / W) ** 2
    return np.where(a >= 0.0, i0(beta * np.sqrt(np.maximum(a, 0.0))), 0.0)


def kb_ft(nu, W: int, beta: float):
    """Continuous Fourier transform of kb_kernel at frequency nu (cycles/cell)."""
    nu = np.asarray(nu, np.float64)
    z2 = beta ** 2 - (math.pi * W * nu) ** 2
    out = np.empty_like(z2)
    pos = z2 > 1e-12
    neg = z2 < -1e-12
    mid = ~(pos | neg)
    z = np.sqrt(np.abs(z2))
    out[pos] = W * np.sinh(z[pos]) / z[pos]
    out[neg] = W * np.sin(z[neg]) / z[neg]
    out[mid] = W
    return out


def grid_size(n: int, sigma: float) -> int:
    G = sigma * n
    if abs(G - round(G)) > 1e-9:
        raise ValueError("sigma * n must be an integer")
    return int(round(G))


class KBGridding:
    """Single-coil gridding NUFFT for an [ny][nx] image and trajectory [M][2]."""

    def __init__(self, traj, ny: int, nx: int, sigma: float = 2.0, W: int = 6):
        if W % 2:
            raise ValueError("W must be even")
        self.traj = np.asarray(traj, np.float64)
        self.ny, self.nx, self.W, self.sigma = ny, nx, W, sigma
        self.Gy, self.Gx = grid_size(ny, sigma), grid_size(nx, sigma)
        self.beta = kb_beta(sigma, W)
        self.iy, self.wy = self._taps(self.traj[:, 0], self.Gy)
        self.ix, self.wx = self._taps(self.traj[:, 1], self.Gx)
        ry = np.arange(ny) - ny // 2
        rx = np.arange(nx) - nx // 2
        self.dy = 1.0 / kb_ft(ry / self.Gy, W, self.beta)
        self.dx = 1.0 / kb_ft(rx / self.Gx, W, self.beta)
        self.scale = 1.0 / math.sqrt(ny * nx)

    def _taps(self, w, G):
        kappa = w * G / (2.0 * math.pi)
        k = np.floor(kappa)[:, None] - self.W // 2 + 1 + np.arange(self.W)[None, :]
        wt = kb_kernel(kappa[:, None] - k, self.W, self.beta)
        return (k.astype(np.int64) % G), wt

    def forward(self, u):
        """[ny][nx] -> [M]."""
        ny, nx = self.ny, self.nx
        g = np.zeros((self.Gy, self.Gx), np.complex128)
        ry = (np.arange(ny) - ny // 2) % self.Gy
        rx = (np.arange(nx) - nx // 2) % self.Gx
        g[np.ix_(ry, rx)] = u * self.dy[:, None] * self.dx[None, :]
        Y = np.fft.fft2(g)
        out = np.zeros(self.traj.shape[0], np.complex128)
        for a in range(self.W):
            for b in range(self.W):
                out += self.wy[:, a] * self.wx[:, b] * Y[self.iy[:, a], self.ix[:, b]]
        return out * self.scale

    def adjoint(self, k):
        """[M] -> [ny][nx], the exact adjoint of forward."""
        Y = np.zeros((self.Gy, self.Gx), np.complex128)
        for a in range(self.W):
            for b in range(self.W):
                np.add.at(Y, (self.iy[:, a], self.ix[:, b]), self.wy[:, a] * self.wx[:, b] * k)
        g = np.fft.ifft2(Y) * (self.Gy * self.Gx)
        ry = (np.arange(self.ny) - self.ny // 2) % self.Gy
        rx = (np.arange(self.nx) - self.nx // 2) % self.Gx
        return g[np.ix_(ry, rx)] * self.dy[:, None] * self.dx[None, :] * self.scale
