"""Pre-whitened SENSE encoding operators, FP64 (oracle side).

Acquisition model b = A~ x + n with n ~ CN(0, Sigma_n) (Sec. 2.1, Eqs. (1)-(2));
pre-whitening with the Cholesky factor L L^H = Sigma_n gives
A = L^-1 A~ and white noise (Sec. 2.1, Eq. (3)).  Because the Fourier
transform and sampling act identically on every channel, L^-1 folds into the
coil maps: S_w,c = sum_d (L^-1)_cd S_d.

Cartesian encoding per coil: A_c x = P . F_c(S_w,c . x), with F_c the centred
orthonormal 2-D DFT (fftshift o fft2 o ifftshift, norm="ortho") and P the
binary sampling mask in centred k-space order.  (The paper does not state the
normalisation or centring; these readings make M = diag(sum_c |s_w,c|^2) at
full sampling and the closed-form SENSE variance exact.)

Normal operator M = A^H A (Sec. 2.1, Eq. (6)).  Everything here is written
out literally, without the separable or folded forms the GPU path uses.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def whiten_maps(maps: np.ndarray, psi: np.ndarray | None) -> np.ndarray:
    """S_w = L^-1 S per pixel, with L = chol(psi) lower (Sec. 2.1, Eq. (3))."""
    maps = np.asarray(maps, np.complex128)
    if psi is None:
        return maps.copy()
    L = np.linalg.cholesky(np.asarray(psi, np.complex128))
    nc = maps.shape[0]
    flat = maps.reshape(nc, -1)
    return sla.solve_triangular(L, flat, lower=True).reshape(maps.shape)


def mask2d(mask: np.ndarray, nx: int) -> np.ndarray:
    """Broadcast a 1-D phase-encode mask [ny] to [ny][nx]; pass 2-D masks through."""
    m = np.asarray(mask)
    if m.ndim == 1:
        m = np.repeat(m[:, None], nx, axis=1)
    return m.astype(np.float64)


def fft2c(x):
    """Centred orthonormal 2-D DFT over the last two axes."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(x, axes=(-2, -1)), norm="ortho"),
                           axes=(-2, -1))


def ifft2c(k):
    """Adjoint (= inverse) of fft2c."""
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(k, axes=(-2, -1)), norm="ortho"),
                           axes=(-2, -1))


class CartesianOp:
    """Whitened Cartesian SENSE encoding A and its normal operator.

    ``maps`` complex [nc][ny][nx] (un-whitened), ``psi`` [nc][nc] or None,
    ``mask`` [ny] (phase-encode lines) or [ny][nx], centred order.
    """

    def __init__(self, maps, psi, mask):
        self.Sw = whiten_maps(maps, psi)
        self.nc, self.ny, self.nx = self.Sw.shape
        self.P = mask2d(mask, self.nx)

    def forward(self, x):
        """A x -> k-space [nc][ny][nx] (zeros off the mask)."""
        return self.P[None] * fft2c(self.Sw * x[None])

    def adjoint(self, y):
        """A^H y -> image [ny][nx]."""
        return np.sum(np.conj(self.Sw) * ifft2c(self.P[None] * y), axis=0)

    def normal(self, x):
        """M x = A^H A x."""
        return self.adjoint(self.forward(x))

    def dense_normal(self):
        """M as a dense N_x x N_x matrix (columns M e_j); tiny grids only."""
        n = self.ny * self.nx
        Md = np.empty((n, n), np.complex128)
        e = np.zeros(n, np.complex128)
        for j in range(n):
            e[:] = 0
            e[j] = 1
            Md[:, j] = self.normal(e.reshape(self.ny, self.nx)).ravel()
        return Md

    def column_normal(self, x_col: int, mask1d: np.ndarray) -> np.ndarray:
        """Dense ny x ny block of M for image column ``x_col`` (1-D masks only).

        With P constant along kx, M = sum_c S_c^H (F_y^H P_y F_y (x) I) S_c is
        block diagonal over image columns; the block is built from the 1-D
        centred orthonormal DFT matrix.
        """
        ny = self.ny
        F = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(np.eye(ny), axes=0), axis=0, norm="ortho"),
                            axes=0)
        C = F.conj().T @ (np.asarray(mask1d, np.float64)[:, None] * F)
        B = np.zeros((ny, ny), np.complex128)
        for c in range(self.nc):
            s = self.Sw[c, :, x_col]
            B += np.conj(s)[:, None] * C * s[None, :]
        return B


def sense_closed_form(maps, psi, ny_R: int):
    """Closed-form SENSE variance and g-factor for uniform 1-D undersampling.

    For a binary mask sampling every R-th phase-encode line (no calibration
    lines) and the orthonormal centred DFT, M is block diagonal over alias
    groups of R pixels spaced ny/R apart in each column.  With the whitened
    Nc x R sensitivity matrix S_g of a group,
        var_acc(m) = R [(S_g^H S_g)^-1]_mm,   var_ref(m) = 1 / [S_g^H S_g]_mm,
        g(m) = sqrt([(S_g^H S_g)^-1]_mm [S_g^H S_g]_mm),
    which is Eq. (11) of Sec. 2.1 evaluated with the classical SENSE
    unfolding (Pruessmann et al. 1999) that the Cartesian experiment uses as
    ground truth (Sec. 3.2.1).  ``ny_R`` is R.
    Returns (var_acc, var_ref, g), each float64 [ny][nx].
    """
    R = int(ny_R)
    Sw = whiten_maps(maps, psi)
    nc, ny, nx = Sw.shape
    assert ny % R == 0
    step = ny // R
    var_acc = np.empty((ny, nx))
    var_ref = np.empty((ny, nx))
    g = np.empty((ny, nx))
    for x in range(nx):
        for y0 in range(step):
            ys = [y0 + m * step for m in range(R)]
            Sg = Sw[:, ys, x]                    # nc x R
            G = Sg.conj().T @ Sg
            Gi = np.linalg.inv(G)
            for m, y in enumerate(ys):
                var_acc[y, x] = R * Gi[m, m].real
                var_ref[y, x] = 1.0 / G[m, m].real
                g[y, x] = np.sqrt(Gi[m, m].real * G[m, m].real)
    return var_acc, var_ref, g


def exact_diag_1d(op: CartesianOp, mask1d, lam: float = 0.0, cols=None):
    """Exact diag(Sigma) for a 1-D mask by dense per-column inversion.

    Sigma = (M + lam I)^-1 M (M + lam I)^-1 (Sec. 2.1, Eq. (8)); lam = 0
    gives M^-1 (Eq. (9)).  Returns float64 [ny][nx] (NaN outside ``cols``).
    """
    ny, nx = op.ny, op.nx
    out = np.full((ny, nx), np.nan)
    cols = range(nx) if cols is None else cols
    for x in cols:
        B = op.column_normal(x, mask1d)
        if lam == 0.0:
            Bi = np.linalg.inv(B)
            out[:, x] = np.real(np.diag(Bi))
        else:
            Ri = np.linalg.inv(B + lam * np.eye(ny))
            out[:, x] = np.real(np.diag(Ri @ B @ Ri))
    return out


def exact_cov_dense(op, lam: float = 0.0):
    """Full Sigma (tiny grids): (M + lam)^-1 M (M + lam)^-1, or M^-1."""
    Md = op.dense_normal()
    n = Md.shape[0]
    if lam == 0.0:
        return np.linalg.inv(Md)
    Ri = np.linalg.inv(Md + lam * np.eye(n))
    return Ri @ Md @ Ri
