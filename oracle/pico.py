"""PICO estimator, covariance application and PMR baseline, FP64 (oracle side).

Image covariance of the linear reconstruction x = R_lam b_w,
R_lam = (M + lam I)^-1 A^H (Sec. 2.1, Eqs. (5), (7)):
    Sigma = (M + lam I)^-1 M (M + lam I)^-1     (Eq. (8)),  Sigma = M^-1 at lam = 0 (Eq. (9)).
Sigma v is applied implicitly as R (R^H v) with CG solves (Sec. 2.2,
"Implicit matrix-vector product via CG"): for lam = 0 one solve of M u = v;
for lam > 0, w = (M + lam)^-1 v, t = M w, u = (M + lam)^-1 t.

Estimator (Sec. 2.2, Eqs. (13)-(14); App. A, Algorithm 1):
    s += conj(v^(i)) . u^(i)   for i = 1..N,    var = Re(s / N).
The imaginary part is kept as a diagnostic (it vanishes in expectation).

Lambda: the paper normalises every forward operator by a 15-step power
method with a 1.01 margin (Sec. 3.3) and states lam for the normalised
operator (Sec. 3.2.2: lam = 0.1).  This oracle keeps the un-normalised
whitened A (maps in units of whitened noise variance) and uses
lam' = lam * 1.01 * lambda_max(M), the same reconstruction up to the image
scale.

PMR (Sec. 1, pseudo multiple replica; App. C): replicas x_r = R_lam n_r with
n_r ~ CN(0, I) white k-space noise; the unbiased sample variance
(sum |x|^2 - |sum x|^2 / N) / (N - 1).  For a linear reconstruction this
equals PMR with data, since f(b + n) - f(b) = R n.
"""
from __future__ import annotations

import numpy as np

from . import philox
from .sense import CartesianOp, fft2c
from .solvers import cg, power_method


class Covariance:
    """Sigma = R R^H for a CG-SENSE reconstruction of ``op``.

    ``lam_rel`` is lam of the normalised operator; ``cg_iters`` CG iterations
    per solve (fixed unless ``tol`` > 0).
    """

    def __init__(self, op, lam_rel: float = 0.0, cg_iters: int = 30, tol: float = 0.0,
                 power_iters: int = 15, margin: float = 1.01):
        self.op = op
        self.shape = (op.ny, op.nx)
        self.cg_iters = cg_iters
        self.tol = tol
        self.lam_rel = lam_rel
        if lam_rel > 0.0:
            self.s2 = power_method(op.normal, self.shape, power_iters, margin)
            self.lam = lam_rel * self.s2
        else:
            self.s2 = None
            self.lam = 0.0

    def solve(self, b):
        """(M + lam)^-1 b by CG."""
        return cg(self.op.normal, b, self.cg_iters, self.lam, self.tol)

    def apply(self, v):
        """u = Sigma v."""
        if self.lam == 0.0:
            return self.solve(v)
        w = self.solve(v)
        t = self.op.normal(w)
        return self.solve(t)

    def recon(self, kspace):
        """x = (M + lam)^-1 A^H y (the CG-SENSE reconstruction itself)."""
        return self.solve(self.op.adjoint(kspace))


def probe_image(seed: int, i: int, shape, dist: str = "phase"):
    """Probe v^(i) as an image; the voxel index is the row-major flat index."""
    n = int(np.prod(shape))
    return philox.probe(seed, i, n, dist).reshape(shape)


def noise_map(cov: Covariance, seed: int, first: int, nprobes: int, dist: str = "phase",
              acc=None, probes=None):
    """Add probes [first, first + nprobes) into the accumulators.

    Returns dict(sum=sum Re(conj v u), sum_im=sum Im(conj v u),
    sumsq=sum (Re(conj v u))^2, count).  ``acc`` continues a previous call.
    ``probes`` (an iterable of images) replaces the Philox draws, for exact
    enumeration over a finite probe distribution.
    """
    shape = cov.shape
    if acc is None:
        acc = {"sum": np.zeros(shape), "sum_im": np.zeros(shape),
               "sumsq": np.zeros(shape), "count": 0}
    if probes is None:
        probes = (probe_image(seed, i, shape, dist) for i in range(first, first + nprobes))
    for v in probes:
        u = cov.apply(v)
        d = np.conj(v) * u
        acc["sum"] += d.real
        acc["sum_im"] += d.imag
        acc["sumsq"] += d.real ** 2
        acc["count"] += 1
    return acc


def noise_map_exact_columns(op, mask1d, seed: int, first: int, nprobes: int, cols,
                            lam: float = 0.0, dist: str = "phase"):
    """Estimator sums with Sigma applied exactly, on selected image columns.

    For a phase-encode mask M is block diagonal over image columns, so
    (Sigma v)[:, x] = Sigma_x v[:, x] with the dense ny x ny block
    Sigma_x = (B_x + lam)^-1 B_x (B_x + lam)^-1 (Sec. 2.1, Eqs. (8)-(9)).
    This is the estimator of Eq. (14) with converged solves; it lets
    full-size problems be checked column by column.  ``lam`` is absolute.
    Returns float64 [ny][len(cols)] of sum_i Re(conj v_i . Sigma v_i).
    """
    ny, nx = op.ny, op.nx
    out = np.zeros((ny, len(cols)))
    V = np.stack([probe_image(seed, i, (ny, nx), dist) for i in range(first, first + nprobes)])
    for j, x in enumerate(cols):
        B = op.column_normal(x, mask1d)
        if lam == 0.0:
            S = np.linalg.inv(B)
        else:
            Ri = np.linalg.inv(B + lam * np.eye(ny))
            S = Ri @ B @ Ri
        vc = V[:, :, x]                       # [N][ny]
        u = vc @ S.T                          # rows: Sigma_x v
        out[:, j] = np.sum((np.conj(vc) * u).real, axis=0)
    return out


def finalize(acc):
    """var = Re(s / N) (App. A, Algorithm 1, last step)."""
    return acc["sum"] / acc["count"]


def pmr_noise(op, seed: int, r: int):
    """White k-space noise replica n_r ~ CN(0, I) for ``op``, zero off the mask.

    Philox element index (c * ny + ky) * nx + x (Cartesian) or c * M + m
    (non-Cartesian, M samples per coil).  For a 1-D phase-encode
    mask the draw is made in the hybrid (ky, x) domain and carried to k-space
    by the centred orthonormal DFT along x; F_x is unitary, so the result is
    still CN(0, I) and the separable GPU path can consume the hybrid draw
    directly.
    """
    if hasattr(op, "traj"):
        # non-Cartesian: element index c * M + m over the acquired samples
        return philox.probe(seed, r, op.nc * op.M, "gaussian",
                            stream=philox.STREAM_PMR).reshape(op.nc, op.M)
    nc, ny, nx = op.nc, op.ny, op.nx
    h = philox.probe(seed, r, nc * ny * nx, "gaussian", stream=philox.STREAM_PMR)
    h = h.reshape(nc, ny, nx)
    if getattr(op, "mask_is_1d", False):
        k = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(h, axes=-1), axis=-1, norm="ortho"),
                            axes=-1)
    else:
        k = h
    return op.P[None] * k


def pmr(cov: Covariance, seed: int, first: int, nrep: int, acc=None):
    """Pseudo multiple replica: accumulate sum x, sum |x|^2 over replicas."""
    shape = cov.shape
    if acc is None:
        acc = {"sum": np.zeros(shape), "sum_im": np.zeros(shape),
               "sumsq": np.zeros(shape), "count": 0}
    for r in range(first, first + nrep):
        n = pmr_noise(cov.op, seed, r)
        x = cov.recon(n)
        acc["sum"] += x.real
        acc["sum_im"] += x.imag
        acc["sumsq"] += np.abs(x) ** 2
        acc["count"] += 1
    return acc


def pmr_finalize(acc):
    """Unbiased sample variance (sum |x|^2 - |sum x|^2 / N) / (N - 1)."""
    N = acc["count"]
    m2 = acc["sum"] ** 2 + acc["sum_im"] ** 2
    return (acc["sumsq"] - m2 / N) / (N - 1)


def cartesian(maps, psi, mask):
    """CartesianOp with the 1-D-mask flag set for the PMR hybrid draw."""
    op = CartesianOp(maps, psi, mask)
    op.mask_is_1d = np.asarray(mask).ndim == 1
    return op


def nrmse_std(var_est, var_ref):
    """NRMSE of standard-deviation maps, ||s - s_ref|| / ||s_ref||.

    The paper computes NRMSE on noise standard-deviation maps (Sec. 3.2.3)
    without printing the formula; this is the plain relative 2-norm over the
    field of view, with s = sqrt(max(var, 0)).
    """
    s = np.sqrt(np.maximum(var_est, 0.0))
    s0 = np.sqrt(np.maximum(var_ref, 0.0))
    return float(np.linalg.norm(s - s0) / np.linalg.norm(s0))


def stderr_proxy(acc):
    """Reference-free estimate of the std-map NRMSE of the running estimate.

    m = sum / N per voxel; the N per-probe terms Re(conj v u) have sample
    variance s2 = (sumsq - N m^2) / (N - 1), so m has variance s2 / N and,
    to first order, sqrt(m) has variance s2 / (4 N m).  The proxy is
    sqrt(sum_k s2_k / (4 N m_k) / sum_k m_k) over voxels with m_k > 0: the
    expected ||sqrt(m) - sigma|| / ||sigma|| (adaptive stopping on the
    per-voxel standard error, Sec. 5, Discussion).
    """
    N = float(acc["count"])
    m = acc["sum"] / N
    s2 = np.maximum((acc["sumsq"] - N * m * m) / (N - 1.0), 0.0)
    pos = m > 0
    return float(np.sqrt(np.sum(s2[pos] / (4.0 * N * m[pos])) / np.sum(m[pos])))


def nrmse_var(var_est, var_ref):
    """NRMSE of variance maps."""
    return float(np.linalg.norm(var_est - var_ref) / np.linalg.norm(var_ref))


def certify(maps_by_n: dict, gold, roi=None, d_nrmse=0.005, d_roi=0.002):
    """Reference-convergence protocol of App. E.

    ``maps_by_n`` maps N -> variance map; ``gold`` is the N_max map.  The
    reference is converged at the smallest N whose doubling (2N present)
    improves NRMSE vs gold by < d_nrmse and changes the ROI-mean variance by
    < d_roi (relative).  Returns that N or None.
    """
    roi = np.ones_like(gold, bool) if roi is None else roi
    for n in sorted(maps_by_n):
        if 2 * n not in maps_by_n:
            continue
        e1 = nrmse_std(maps_by_n[n], gold)
        e2 = nrmse_std(maps_by_n[2 * n], gold)
        r1 = maps_by_n[n][roi].mean()
        r2 = maps_by_n[2 * n][roi].mean()
        if (e1 - e2) < d_nrmse and abs(r2 - r1) / abs(r2) < d_roi:
            return n
    return None


__all__ = ["Covariance", "noise_map", "noise_map_exact_columns", "finalize", "pmr", "pmr_finalize", "pmr_noise",
           "probe_image", "cartesian", "nrmse_std", "nrmse_var", "certify", "fft2c"]
