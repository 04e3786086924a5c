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


# ---------------------------------------------------------------- TV model
# The paper's CS reconstruction (Sec. 3.2.3) penalises lam_TV ||grad x||_1 and
# runs FISTA; it does not say how the TV proximal step is computed.  Readings:
# isotropic TV of the complex image, TV(x) = sum_r sqrt(|D_y x|_r^2 + |D_x x|_r^2),
# forward differences with periodic wrap (D_y x[y] = x[y+1] - x[y]); the
# proximal step prox_{lam TV}(z) by the fast gradient projection on the dual
# (Beck and Teboulle, IEEE TIP 2009): p, r in C^{2 x ny x nx}, from r = p = 0,
#     w = r + (1 / (8 lam)) D (z - lam D^H r),  p' = P(w),
#     r' = p' + ((s - 1) / s') (p' - p),  s' = (1 + sqrt(1 + 4 s^2)) / 2,
# with P the per-pixel projection onto {|p_y|^2 + |p_x|^2 <= 1}, for a fixed
# number of inner iterations, and x = z - lam D^H p.  The reconstruction map
# is then a composition of steps differentiable almost everywhere; its
# forward-mode derivative runs through the unrolled inner iterations (what
# automatic differentiation of such an implementation evaluates), with
# dP(w) dw = dw for |w| <= 1 and (dw - w^ Re(w^H dw)) / |w| otherwise.


def tv_grad(x):
    """D x: forward differences along y and x, periodic; shape (2, ny, nx)."""
    return np.stack([np.roll(x, -1, axis=-2) - x, np.roll(x, -1, axis=-1) - x])


def tv_grad_adj(p):
    """D^H p (the negative divergence): p_y[y-1] - p_y[y] + p_x[x-1] - p_x[x]."""
    return (np.roll(p[0], 1, axis=-2) - p[0]) + (np.roll(p[1], 1, axis=-1) - p[1])


def ball_proj(w):
    n = np.sqrt(np.abs(w[0]) ** 2 + np.abs(w[1]) ** 2)
    return w / np.maximum(n, 1.0)


def ball_dproj(w, dw):
    n = np.sqrt(np.abs(w[0]) ** 2 + np.abs(w[1]) ** 2)
    out = np.array(dw, copy=True)
    big = n > 1.0
    if np.any(big):
        wh = w[:, big] / n[big]
        re = np.real(np.conj(wh[0]) * dw[0][big] + np.conj(wh[1]) * dw[1][big])
        out[:, big] = (dw[:, big] - wh * re) / n[big]
    return out


def tv_prox(z, lam, inner):
    """prox_{lam TV}(z) by ``inner`` dual fast-gradient-projection steps from zero."""
    if lam == 0.0:
        return np.array(z, copy=True)
    p = np.zeros((2,) + z.shape, np.complex128)
    r = p.copy()
    s = 1.0
    for _ in range(inner):
        w = r + tv_grad(z - lam * tv_grad_adj(r)) / (8.0 * lam)
        pn = ball_proj(w)
        sn = (1.0 + np.sqrt(1.0 + 4.0 * s * s)) / 2.0
        r = pn + ((s - 1.0) / sn) * (pn - p)
        p, s = pn, sn
    return z - lam * tv_grad_adj(p)


def tv_dprox(z, dz, lam, inner):
    """Forward-mode derivative of tv_prox at z applied to dz (same iterations)."""
    if lam == 0.0:
        return np.array(dz, copy=True)
    p = np.zeros((2,) + z.shape, np.complex128)
    r, dp, dr = p.copy(), p.copy(), p.copy()
    s = 1.0
    for _ in range(inner):
        w = r + tv_grad(z - lam * tv_grad_adj(r)) / (8.0 * lam)
        dw = dr + tv_grad(dz - lam * tv_grad_adj(dr)) / (8.0 * lam)
        pn, dpn = ball_proj(w), ball_dproj(w, dw)
        sn = (1.0 + np.sqrt(1.0 + 4.0 * s * s)) / 2.0
        th = (s - 1.0) / sn
        r, dr = pn + th * (pn - p), dpn + th * (dpn - dp)
        p, dp, s = pn, dpn, sn
    return dz - lam * tv_grad_adj(dp)


class FistaTV:
    """T-iteration FISTA with the TV proximal step and its forward-mode Jacobian.

    Same outer iteration, step and normalisation as FistaL1Wavelet; the
    proximal step is tv_prox(z_k, lam, inner).  ``recon(store=True)`` keeps
    z_k, from which ``jvp`` recomputes each inner trajectory.
    """

    def __init__(self, op, lam: float, iters: int = 100, inner: int = 10, power_iters: int = 15,
                 margin: float = 1.01):
        self.op = op
        self.lam = lam
        self.T = iters
        self.inner = inner
        self.shape = (op.ny, op.nx)
        self.s2 = power_method(op.normal, self.shape, power_iters, margin)
        t = [1.0]
        for _ in range(iters):
            t.append((1.0 + np.sqrt(1.0 + 4.0 * t[-1] ** 2)) / 2.0)
        self.t = t

    def theta(self, k):
        return (self.t[k - 1] - 1.0) / self.t[k]

    def recon(self, b, store=False):
        atb = self.op.adjoint(b)
        x_prev = np.zeros(self.shape, np.complex128)
        y = x_prev.copy()
        zs = []
        for k in range(1, self.T + 1):
            z = y - (self.op.normal(y) - atb) / self.s2
            if store:
                zs.append(z)
            x = tv_prox(z, self.lam, self.inner)
            y = x + self.theta(k) * (x - x_prev)
            x_prev = x
        return (x_prev, zs) if store else x_prev

    def jvp(self, w, zs):
        g = self.op.adjoint(w)
        x_prev = np.zeros(self.shape, np.complex128)
        y = x_prev.copy()
        for k in range(1, self.T + 1):
            dz = y - (self.op.normal(y) - g) / self.s2
            x = tv_dprox(zs[k - 1], dz, self.lam, self.inner)
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


def noise_map_jvp(fista, cs, seed: int, first: int, nprobes: int,
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
