"""Pins of the oracle's non-Cartesian operators.

  * On a grid-aligned trajectory the direct NUDFT equals the centred
    orthonormal 2-D DFT (library FFT) — a special case fixed by the reading
    of the NUDFT sign and scale.
  * Adjointness of the NUDFT pair.
  * Toeplitz normal operator == NUDFT forward-then-adjoint to rounding.
  * The embedded kernel's DFT is real (Hermitian PSF).
  * M Hermitian PSD; full sampling of every grid point gives M = diag(|s|^2).
"""
import numpy as np

import workloads
from oracle import nufft, pico, sense


def _small(n=16, nc=3, R=1, seed=0, inter=8, samples=64):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n, n, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    traj = workloads.spiral_traj(n, R, inter, samples)
    return maps, psi, traj


def test_grid_aligned_nudft_is_centred_dft():
    n = 12
    ky, kx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    traj = np.stack([2 * np.pi * ky.ravel() / n, 2 * np.pi * kx.ravel() / n], axis=1)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = nufft.nudft_forward(u, traj).reshape(n, n)
    assert np.allclose(a, sense.fft2c(u), atol=1e-12)


def test_nudft_adjointness():
    _, _, traj = _small()
    rng = np.random.default_rng(2)
    u = rng.standard_normal((16, 12)) + 1j * rng.standard_normal((16, 12))
    k = rng.standard_normal(traj.shape[0]) + 1j * rng.standard_normal(traj.shape[0])
    lhs = np.vdot(nufft.nudft_forward(u, traj), k)
    rhs = np.vdot(u, nufft.nudft_adjoint(k, traj, (16, 12)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_toeplitz_equals_nudft_normal_and_kernel_real():
    maps, psi, traj = _small(R=2)
    op = nufft.NonCartOp(maps, psi, traj)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    a = op.normal(x)
    b = op.normal_nudft(x)
    assert np.linalg.norm(a - b) < 1e-12 * np.linalg.norm(b)
    Md = op.dense_normal()
    assert np.allclose(Md, Md.conj().T, atol=1e-12)
    assert np.linalg.eigvalsh(Md).min() > -1e-10


def test_full_grid_sampling_gives_diagonal_normal_operator():
    n, nc = 8, 2
    rng = np.random.default_rng(4)
    maps = workloads.coil_maps(n, n, nc, rng)
    ky, kx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    traj = np.stack([2 * np.pi * ky.ravel() / n, 2 * np.pi * kx.ravel() / n], axis=1)
    op = nufft.NonCartOp(maps, None, traj)
    d = np.sum(np.abs(maps) ** 2, axis=0).ravel()
    assert np.allclose(op.dense_normal(), np.diag(d), atol=1e-12)


def test_noncart_noise_map_enumeration_exact():
    # QPSK enumeration on a 2x2 image through the Toeplitz covariance
    maps, psi, traj = _small(n=4, nc=2, R=2, inter=6, samples=16)
    maps = maps[:, 1:3, 1:3].copy()
    op = nufft.NonCartOp(maps, psi, traj)
    cov = pico.Covariance(op, 0.2, cg_iters=12)
    Md = op.dense_normal()
    Ri = np.linalg.inv(Md + cov.lam * np.eye(4))
    Sig = Ri @ Md @ Ri
    import itertools
    probes = (np.array(c, np.complex128).reshape(2, 2)
              for c in itertools.product([1, 1j, -1, -1j], repeat=4))
    acc = pico.noise_map(cov, 0, 0, 0, probes=probes)
    assert np.allclose(pico.finalize(acc).ravel(), np.real(np.diag(Sig)), rtol=1e-9)
