"""Compressed-sensing reconstruction and its Jacobian probes, FP64 (oracle side).

Reconstruction (Sec. 3.2.3 uses FISTA with standard momentum, Beck and
Teboulle 2009, 100 iterations; Sec. 3.3 normalises every forward operator by
a 15-step power method with a 1.01 margin).  The workload's regulariser is
an L1 penalty on an orthonormal 4-level db4 wavelet transform Psi:

    min_x 1/2 ||A x - b||^2 + lam ||Psi x||_1     (lam of the normalised problem)

With the normalised operator A / s (s^2 = 1.01 lambda_max(A^H A)) the FISTA
step is 1, which for the un-normalised whitened A reads
    z_k = y_k - (M y_k - A^H b) / s^2
    x_k = Psi^H soft_lam(Psi z_k)         (detail coefficients only)
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
    y_{k+1} = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}),
from x_0 = y_1 = 0, t_1 = 1.  soft_lam(c) = c max(0, 1 - lam/|c|) for complex c.

Noise model (Sec. 2.2, "Extension to Compressed-Sensing reconstructions"):
the image covariance is approximated by J J^H with J the Jacobian of the
reconstruction map at the measured data, and the variance map is the mean of
|J w|^2 over probes w (the paper evaluates J w by automatic
differentiation).  Readings: w is a random-phase probe in (whitened)
k-space on the sampled locations, E[w w^H] = I there, so
E|(J w)_k|^2 = (J J^H)_kk; J w is the exact forward-mode derivative of the
T-iteration FISTA map, with the derivative of complex soft-thresholding at
c (|c| > lam):  d = dc - (lam/|c|) c^ j Im(conj(c^) dc), c^ = c/|c|,  and 0
for |c| <= lam (the radial component passes, the tangential one shrinks by
1 - lam/|c|); for lam = 0 the derivative is the identity.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .solvers import power_method
from .wavelet import detail_mask, wavedec2, waverec2


def soft(c, lam, mask):
    a = np.abs(c)
    scale = np.where(a > lam, 1.0 - lam / np.where(a > 0, a, 1.0), 0.0)
    return np.where(mask, c * scale, c)


def dsoft(c, dc, lam, mask):
    """Derivative of soft_lam at c applied to dc (R-linear).

    Active where |c| > lam; at the kink |c| = lam the map has no derivative
    and the coefficient is taken as inactive, except for lam = 0, where
    soft_0 is the identity and differentiable everywhere.
    """
    if lam == 0.0:
        return dc
    a = np.abs(c)
    act = a > lam
    ch = np.where(act, c / np.where(a > 0, a, 1.0), 0.0)
    tang = 1j * ch * np.imag(np.conj(ch) * dc)
    d = np.where(act, dc - (lam / np.where(a > 0, a, 1.0)) * tang, 0.0)
    return np.where(mask, d, dc)


class FistaL1Wavelet:
    """The T-iteration FISTA reconstruction map and its forward-mode Jacobian."""

    def __init__(self, op, lam: float, iters: int = 100, levels: int = 4,
                 power_iters: int = 15, margin: float = 1.01):
        self.op = op
        self.lam = lam
        self.T = iters
        self.levels = levels
        self.shape = (op.ny, op.nx)
        self.s2 = power_method(op.normal, self.shape, power_iters, margin)
        self.mask = detail_mask(self.shape, levels)
        t = [1.0]
        for _ in range(iters):
            t.append((1.0 + np.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
        self.t = t                                   # t_1 .. t_{T+1}

    def theta(self, k):
        """Momentum weight (t_k - 1) / t_{k+1} for k = 1..T."""
        return (self.t[k - 1] - 1.0) / self.t[k]

    def recon(self, b, store=False):
        """x_T (and the coefficients c_k = Psi z_k when store)."""
        atb = self.op.adjoint(b)
        x_prev = np.zeros(self.shape, np.complex128)
        y = x_prev.copy()
        cs = []
        for k in range(1, self.T + 1):
            z = y - (self.op.normal(y) - atb) / self.s2
            c = wavedec2(z, self.levels)
            if store:
                cs.append(c)
            x = waverec2(soft(c, self.lam, self.mask), self.levels)
            y = x + self.theta(k) * (x - x_prev)
            x_prev = x
        return (x_prev, cs) if store else x_prev

    def jvp(self, w, cs):
        """J w at the data whose FISTA coefficients are ``cs`` (recon(store=True))."""
        g = self.op.adjoint(w)
        x_prev = np.zeros(self.shape, np.complex128)
        y = x_prev.copy()
        for k in range(1, self.T + 1):
            z = y - (self.op.normal(y) - g) / self.s2
            dc = dsoft(cs[k - 1], wavedec2(z, self.levels), self.lam, self.mask)
            x = waverec2(dc, self.levels)
            y = x + self.theta(k) * (x - x_prev)
            x_prev = x
        return x_prev


def pmr_cs(fista: FistaL1Wavelet, bw, seed: int, first: int, nrep: int, sigma: float, x0=None,
           acc=None):
    """Pseudo multiple replica for the nonlinear reconstruction (Sec. 1, App. C;
    Sec. 3.2.3 compares it with the Jacobian probes).

    Replica r reconstructs the perturbed whitened data b + sigma n_r, n_r the
    CN(0, I) k-space noise of oracle.pico.pmr_noise (Philox stream 1, element
    (c ny + ky) nx + kx, zero off the mask), and accumulates
    d_r = (x_r - x_0) / sigma with x_0 = f(b): sum Re d, sum Im d, sum |d|^2.
    The unbiased sample variance of d (oracle.pico.pmr_finalize) is the
    replica estimate of diag(J J^H); subtracting x_0 leaves it unchanged and
    keeps the sums well conditioned.
    """
    from .pico import pmr_noise
    if x0 is None:
        x0 = fista.recon(bw)
    shape = fista.shape
    if acc is None:
        acc = {"sum": np.zeros(shape), "sum_im": np.zeros(shape), "sumsq": np.zeros(shape), "count": 0}
    for r in range(first, first + nrep):
        n = pmr_noise(fista.op, seed, r)
        d = (fista.recon(bw + sigma * n) - x0) / sigma
        acc["sum"] += d.real
        acc["sum_im"] += d.imag
        acc["sumsq"] += np.abs(d) ** 2
        acc["count"] += 1
    return acc


def kspace_probe(op, seed: int, i: int, dist: str = "phase"):
    """Probe w^(i) in whitened k-space on the sampled locations.

    Philox element index (c * ny + ky) * nx + kx (centred order), stream 2.
    """
    nc, ny, nx = op.nc, op.ny, op.nx
    w = philox.probe(seed, i, nc * ny * nx, dist, stream=philox.STREAM_JVP).reshape(nc, ny, nx)
    return op.P[None] * w


def noise_map_jvp(fista: FistaL1Wavelet, cs, seed: int, first: int, nprobes: int,
                  dist: str = "phase", acc=None):
    """Accumulate |J w|^2 (sum) and Re/Im of J w over probes."""
    shape = fista.shape
    if acc is None:
        acc = {"sum": np.zeros(shape), "sum_re": np.zeros(shape), "sum_im": np.zeros(shape),
               "count": 0}
    for i in range(first, first + nprobes):
        u = fista.jvp(kspace_probe(fista.op, seed, i, dist), cs)
        acc["sum"] += np.abs(u) ** 2
        acc["sum_re"] += u.real
        acc["sum_im"] += u.imag
        acc["count"] += 1
    return acc
