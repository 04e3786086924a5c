"""Seeded synthetic workloads for the PICO noise-map path.

This module only draws inputs: coil sensitivity maps, channel noise
covariances, Cartesian sampling masks, spiral trajectories, Poisson-disc
masks and a numerical phantom.  It holds none of the method's arithmetic
(no whitening, no Fourier operators, no solver), so that both the FP64
oracle and the GPU library can be fed the very same arrays.

The paper's data sets (Stanford knee, GE spiral phantom, fastMRI knee; Sec. 3.1)
are not available; these generators stand in for them with the same matrix
sizes, channel counts, acceleration factors and calibration regions
(Sec. 3.1-3.2).  No data-set item is reproduced.

Every draw uses ``numpy.random.default_rng(seed)`` in a fixed order, except
the Poisson-disc dart throwing, which runs in C (poisson_disc.c, built with
gcc on first use) on a SplitMix64 stream seeded by ``seed``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "coil_maps", "noise_cov", "cart_mask_1d", "cart_mask_2d_uniform",
    "spiral_traj", "poisson_disc_mask", "phantom", "Problem", "config",
    "CONFIGS",
]


def coil_maps(ny: int, nx: int, nc: int, rng: np.random.Generator) -> np.ndarray:
    """Smooth complex Gaussian-profile receive maps, complex128 [nc][ny][nx].

    Per coil, in this order: ring angle 2*pi*c/nc + U(-0.2, 0.2), ring radius
    U(0.4, 0.6) (the profile centre), width U(0.3, 0.6) FOV, phase-ramp
    slopes a, b ~ U(-1, 1) cycles/FOV, phase offset U(0, 2*pi).  No RSS
    normalisation.
    """
    yy = (np.arange(ny) - ny / 2) / ny
    xx = (np.arange(nx) - nx / 2) / nx
    y, x = np.meshgrid(yy, xx, indexing="ij")
    out = np.empty((nc, ny, nx), np.complex128)
    for c in range(nc):
        ang = 2 * math.pi * c / nc + rng.uniform(-0.2, 0.2)
        rad = rng.uniform(0.4, 0.6)
        w = rng.uniform(0.3, 0.6)
        a = rng.uniform(-1.0, 1.0)
        b = rng.uniform(-1.0, 1.0)
        phi = rng.uniform(0.0, 2 * math.pi)
        cy, cx = rad * math.sin(ang), rad * math.cos(ang)
        mag = np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * w * w))
        out[c] = mag * np.exp(1j * (phi + 2 * math.pi * (a * x + b * y)))
    return out


def noise_cov(nc: int, rng: np.random.Generator) -> np.ndarray:
    """Random Hermitian positive-definite channel covariance, complex128 [nc][nc].

    Psi = D^1/2 C D^1/2 with d_c ~ U(0.5, 2) and C Hermitian with unit
    diagonal.  Off-diagonal |rho| ~ U(0.1, 0.3) with uniform phase for every
    pair when nc <= 4; otherwise for ring neighbours, U(0.05, 0.15) at ring
    distance 2 and 0 beyond (diagonal dominance keeps C positive definite).
    """
    d = rng.uniform(0.5, 2.0, size=nc)
    C = np.eye(nc, dtype=np.complex128)
    for i in range(nc):
        for j in range(i + 1, nc):
            if nc <= 4:
                lo, hi = 0.1, 0.3
            else:
                dist = min(j - i, nc - (j - i))
                if dist == 1:
                    lo, hi = 0.1, 0.3
                elif dist == 2:
                    lo, hi = 0.05, 0.15
                else:
                    continue
            mag = rng.uniform(lo, hi)
            ph = rng.uniform(0.0, 2 * math.pi)
            C[i, j] = mag * np.exp(1j * ph)
            C[j, i] = np.conj(C[i, j])
    s = np.sqrt(d)
    return (s[:, None] * C) * s[None, :]


def cart_mask_1d(ny: int, R: int, acs: int = 0) -> np.ndarray:
    """Phase-encode mask, uint8 [ny], in centred k-space order.

    Line j is sampled iff (j - ny/2) mod R == 0; with ``acs`` > 0 the lines
    [ny/2 - acs/2, ny/2 + acs/2) are sampled too (Sec. 3.2.1 uses uniform R=2;
    Sec. 3.1 a 24-line calibration region).
    """
    j = np.arange(ny)
    m = ((j - ny // 2) % R == 0)
    if acs:
        m |= (j >= ny // 2 - acs // 2) & (j < ny // 2 + acs // 2)
    return m.astype(np.uint8)


def cart_mask_2d_uniform(ny: int, nx: int, Ry: int, Rx: int = 1) -> np.ndarray:
    """Separable uniform mask, uint8 [ny][nx] (centred order)."""
    my = ((np.arange(ny) - ny // 2) % Ry == 0)
    mx = ((np.arange(nx) - nx // 2) % Rx == 0)
    return (my[:, None] & mx[None, :]).astype(np.uint8)


def spiral_traj(n: int, R: int = 1, interleaves: int = 48, samples: int = 4096) -> np.ndarray:
    """Variable-density multi-interleave spiral, float64 [M][2] = (w_y, w_x) in rad.

    r(t) = kmax t^1.5 cycles/FOV with kmax = n/2 - 0.5, phi = 2 pi T t + 2 pi l/L,
    T = ceil(1.5 kmax / L) turns, t = s/(S-1).  Interleave subsampling keeps
    l = 0 (mod R) (Sec. 3.2.2).  w = 2 pi k / n, so |w| < pi.
    """
    kmax = n / 2 - 0.5
    turns = math.ceil(kmax * 1.5 / interleaves)
    t = np.arange(samples) / (samples - 1)
    r = kmax * t ** 1.5
    out = []
    for l in range(0, interleaves, R):
        phi = 2 * math.pi * turns * t + 2 * math.pi * l / interleaves
        ky = r * np.sin(phi)
        kx = r * np.cos(phi)
        out.append(np.stack([2 * math.pi * ky / n, 2 * math.pi * kx / n], axis=1))
    return np.concatenate(out, axis=0)


_PD_LIB = None


def _pd_lib():
    """The C dart-throwing sampler (poisson_disc.c), built with gcc on first use."""
    global _PD_LIB
    if _PD_LIB is not None:
        return _PD_LIB
    import ctypes
    import os
    import subprocess
    import tempfile
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "poisson_disc.c")
    so = os.path.join(here, "_poisson_disc.so")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        fd, tmp = tempfile.mkstemp(suffix=".so", dir=here)
        os.close(fd)
        subprocess.run(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"], check=True)
        os.replace(tmp, so)
    lib = ctypes.CDLL(so)
    lib.poisson_disc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_void_p]
    lib.poisson_disc.restype = ctypes.c_int
    _PD_LIB = lib
    return lib


def _poisson_disc(ny: int, nx: int, r0: float, calib: int, seed: int, k: int = 30) -> np.ndarray:
    """Bridson dart throwing with radius r(k) = r0 (1 + 2 |k| / kmax), plus the
    calib x calib fully sampled centre."""
    m = np.zeros((ny, nx), np.uint8)
    if _pd_lib().poisson_disc(ny, nx, float(r0), k, seed & (2**64 - 1), m.ctypes.data) < 0:
        raise MemoryError("poisson_disc")
    m[ny // 2 - calib // 2: ny // 2 + calib // 2, nx // 2 - calib // 2: nx // 2 + calib // 2] = 1
    return m


def poisson_disc_mask(ny: int, nx: int, R: float, calib: int, seed: int,
                      tol: float = 0.01) -> np.ndarray:
    """Variable-density Poisson-disc mask, uint8 [ny][nx] (centred order).

    r0 is bisected until the sampled fraction is 1/R within ``tol``
    (relative), the calib x calib centre included (Sec. 3.2.3).
    """
    lo, hi = 0.3, 4.0
    best = None
    for _ in range(30):
        r0 = 0.5 * (lo + hi)
        m = _poisson_disc(ny, nx, r0, calib, seed)
        acc = m.size / m.sum()
        best = m
        if abs(acc - R) <= tol * R:
            break
        if acc < R:
            lo = r0
        else:
            hi = r0
    return best


def phantom(n: int, rng: np.random.Generator, ellipses: int = 12) -> np.ndarray:
    """Complex ellipse phantom, complex128 [n][n], max |x| = 1.

    ``ellipses`` seeded ellipses (centre U(-0.35, 0.35), semi-axes
    U(0.05, 0.35), angle U(0, pi), additive intensity U(-0.3, 1)), clipped at
    0, times the smooth phase exp(j pi (0.5 x + 0.3 y + 0.2 x y)).
    """
    yy = (np.arange(n) - n / 2) / n
    y, x = np.meshgrid(yy, yy, indexing="ij")
    img = np.zeros((n, n))
    for _ in range(ellipses):
        cy, cx = rng.uniform(-0.35, 0.35, size=2)
        ay, ax = rng.uniform(0.05, 0.35, size=2)
        th = rng.uniform(0, math.pi)
        val = rng.uniform(-0.3, 1.0)
        c, s = math.cos(th), math.sin(th)
        u = (x - cx) * c + (y - cy) * s
        v = -(x - cx) * s + (y - cy) * c
        img += val * ((u / ax) ** 2 + (v / ay) ** 2 <= 1)
    img = np.clip(img, 0, None)
    z = img * np.exp(1j * math.pi * (0.5 * x + 0.3 * y + 0.2 * x * y))
    return z / np.abs(z).max()


@dataclass
class Problem:
    """One noise-map problem: the encoding inputs plus the solver settings."""
    name: str
    ny: int
    nx: int
    maps: np.ndarray                 # complex128 [nc][ny][nx], un-whitened
    psi: np.ndarray                  # complex128 [nc][nc]
    sampling: str                    # "cart1d" | "cart2d" | "noncart"
    mask: np.ndarray | None = None   # uint8 [ny] or [ny][nx], centred order
    traj: np.ndarray | None = None   # float64 [M][2] (w_y, w_x)
    lam: float = 0.0                 # Tikhonov weight, relative to the normalised operator
    cg_iters: int = 20
    probes: int = 16
    recon: str = "cgsense"           # "cgsense" | "cs"
    extra: dict = field(default_factory=dict)

    @property
    def nc(self) -> int:
        return self.maps.shape[0]


def config(i: int, seed: int = 0, **kw) -> Problem:
    """Problem for workload i (1-based), seeded.

    1: 64x64, 4 coils, R=2 uniform 1-D, 16 probes, CG 20 its, lambda 0.
    2: 320x320, 15 coils, R=2 uniform + 24 centre lines, 256 probes, CG 30 its.
    3: spiral 256x256, 16 coils, 48x4096 interleaves subsampled by R (kw R=2),
       lambda 0.1, CG 30 its, 256 probes.
    4: 320x320 CS, 8 coils, Poisson-disc R=2 with 24x24 calibration, 128 probes,
       L1-db4 FISTA 100 its, lambda 1e-3; with reg="tv" the model of the paper's
       CS experiment (Sec. 3.2.3): 15 coils, TV weight 1e-2, 10 dual steps per
       proximal step.
    Keyword overrides: ny, nx, nc, R, acs, probes, cg_iters, lam (and for 4:
    calib, fista_iters, cs_lambda, snr_db, reg, tv_inner).
    """
    rng = np.random.default_rng(seed)
    if i == 1:
        ny = kw.get("ny", 64); nx = kw.get("nx", 64); nc = kw.get("nc", 4)
        maps = coil_maps(ny, nx, nc, rng)
        psi = noise_cov(nc, rng)
        mask = cart_mask_1d(ny, kw.get("R", 2), kw.get("acs", 0))
        return Problem("cart1d-64-4c-R2", ny, nx, maps, psi, "cart1d", mask=mask,
                       lam=kw.get("lam", 0.0), cg_iters=kw.get("cg_iters", 20),
                       probes=kw.get("probes", 16))
    if i == 2:
        ny = kw.get("ny", 320); nx = kw.get("nx", 320); nc = kw.get("nc", 15)
        maps = coil_maps(ny, nx, nc, rng)
        psi = noise_cov(nc, rng)
        mask = cart_mask_1d(ny, kw.get("R", 2), kw.get("acs", 24))
        return Problem(f"cart1d-{ny}x{nx}-{nc}c-R2-acs", ny, nx, maps, psi, "cart1d",
                       mask=mask, lam=kw.get("lam", 0.0), cg_iters=kw.get("cg_iters", 30),
                       probes=kw.get("probes", 256))
    if i == 3:
        n = kw.get("ny", 256); nc = kw.get("nc", 16); R = kw.get("R", 2)
        maps = coil_maps(n, n, nc, rng)
        psi = noise_cov(nc, rng)
        traj = spiral_traj(n, R, kw.get("interleaves", 48), kw.get("samples", 4096))
        return Problem(f"spiral-{n}-{nc}c-R{R}", n, n, maps, psi, "noncart", traj=traj,
                       lam=kw.get("lam", 0.1), cg_iters=kw.get("cg_iters", 30),
                       probes=kw.get("probes", 256),
                       extra={"oversamp": kw.get("oversamp", 2.0), "kb_width": kw.get("kb_width", 6)})
    if i == 4:
        tv = kw.get("reg", "l1wav") == "tv"
        n = kw.get("ny", 320); nc = kw.get("nc", 15 if tv else 8)
        maps = coil_maps(n, n, nc, rng)
        psi = noise_cov(nc, rng)
        x = phantom(n, rng)
        mask = poisson_disc_mask(n, n, kw.get("R", 2.0), kw.get("calib", 24), seed)
        return Problem(f"cs-{'tv' if tv else 'l1wav'}-{n}-{nc}c", n, n, maps, psi, "cart2d", mask=mask,
                       recon="cs", probes=kw.get("probes", 128),
                       extra={"phantom": x, "fista_iters": kw.get("fista_iters", 100),
                              "cs_lambda": kw.get("cs_lambda", 1e-2 if tv else 1e-3), "levels": 4,
                              "snr_db": kw.get("snr_db", 45.0), "reg": "tv" if tv else "l1wav",
                              "tv_inner": kw.get("tv_inner", 10)})
    raise ValueError(f"unknown workload {i}")


CONFIGS = {
    1: "2D Cartesian SENSE 64x64, 4 coils, R=2 uniform, 16 random-phase probes, CG 20 its",
    2: "2D Cartesian SENSE 320x320 complex64, 15 coils, R=2 + 24 ACS lines, K=256 probes, CG 30 its",
    3: "spiral 256x256, 16 coils, 48x4096 interleaves subsampled R=2/3/4, lambda 0.1, K=256, CG 30 its",
    4: "CS 320x320, 8 coils, Poisson-disc R=2 (24x24 calib), L1-db4 FISTA 100 its, K=128 JVP probes",
}
