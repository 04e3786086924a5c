"""Pins of the oracle's Kaiser-Bessel gridding NUFFT: the Bessel series
against scipy's library routine, the closed-form kernel transform against
numerical quadrature, gridding against the direct NUDFT within the kernel's
error (falling with the width), and exact adjointness."""
import math

import numpy as np
import pytest
from scipy import integrate, special

import workloads
from oracle import kbnufft as kb
from oracle import nufft


def test_i0_series_matches_library():
    x = np.linspace(0.0, 20.0, 81)
    np.testing.assert_allclose(kb.i0(x), special.i0(x), rtol=1e-14)


@pytest.mark.parametrize("sigma,W", [(2.0, 6), (1.25, 4), (2.0, 4)])
def test_kernel_transform_closed_form(sigma, W):
    beta = kb.kb_beta(sigma, W)
    for nu in (0.0, 0.05, 0.13, 0.25, 0.4, 0.6, 0.9):
        re, _ = integrate.quad(lambda u: float(kb.kb_kernel(u, W, beta)) * math.cos(2 * math.pi * nu * u),
                               -W / 2, W / 2, epsabs=0, epsrel=1e-11, limit=400)
        assert kb.kb_ft(np.array([nu]), W, beta)[0] == pytest.approx(re, rel=1e-9)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_gridding_approximates_nudft():
    n = 48
    traj = workloads.spiral_traj(n, 2, 12, 300)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = nufft.nudft_forward(u, traj)
    errs = {}
    for sigma, W in ((2.0, 2), (2.0, 4), (2.0, 6), (1.25, 4)):
        g = kb.KBGridding(traj, n, n, sigma, W)
        errs[(sigma, W)] = _rel(g.forward(u), ref)
        # adjoint against the NUDFT adjoint, same bound
        k = rng.standard_normal(traj.shape[0]) + 1j * rng.standard_normal(traj.shape[0])
        ea = _rel(g.adjoint(k), nufft.nudft_adjoint(k, traj, (n, n)))
        assert ea < 3 * errs[(sigma, W)] + 1e-12
    assert errs[(2.0, 6)] < 1e-5
    assert errs[(2.0, 4)] < 1e-3
    assert errs[(1.25, 4)] < 2e-2
    assert errs[(2.0, 6)] < errs[(2.0, 4)] < errs[(2.0, 2)]


def test_gridding_adjointness_and_taps():
    ny, nx = 32, 40
    traj = workloads.spiral_traj(40, 1, 8, 200)
    g = kb.KBGridding(traj, ny, nx, 2.0, 6)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    k = rng.standard_normal(traj.shape[0]) + 1j * rng.standard_normal(traj.shape[0])
    lhs = np.vdot(k, g.forward(u))
    rhs = np.vdot(g.adjoint(k), u)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # every tap lies within W/2 cells of its sample (modulo the grid)
    kappa = traj[:, 0] * g.Gy / (2 * math.pi)
    d = (kappa[:, None] - g.iy + g.Gy / 2) % g.Gy - g.Gy / 2
    assert np.all(np.abs(d) <= g.W / 2 + 1e-9)


@pytest.mark.parametrize("sigma,W,bound", [(2.0, 6, 1e-5), (1.25, 4, 1e-2)])
def test_gridding_normal_operator(sigma, W, bound):
    # M_grid = sum_c S^H A_grid^H A_grid S against the exact (Toeplitz = NUDFT)
    # normal operator: within the gridding error, which falls with the width;
    # Hermitian and positive by construction (A_grid^H is the exact adjoint)
    n = 32
    rng = np.random.default_rng(7)
    maps = workloads.coil_maps(n, n, 3, rng)
    psi = workloads.noise_cov(3, rng)
    traj = workloads.spiral_traj(n, 2, 12, 400)
    exact = nufft.NonCartOp(maps, psi, traj)
    grid = nufft.NonCartOp(maps, psi, traj, kb=(sigma, W), normal_mode="gridding")
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    mg, mt = grid.normal(x), exact.normal(x)
    e = _rel(mg, mt)
    assert 1e-12 < e < bound
    np.testing.assert_allclose(mg, grid.normal_gridding(x), rtol=0, atol=0)
    lhs, rhs = np.vdot(y, grid.normal(x)), np.vdot(grid.normal(y), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert np.vdot(x, mg).real > 0 and abs(np.vdot(x, mg).imag) <= 1e-12 * abs(np.vdot(x, mg))
    with pytest.raises(ValueError):
        nufft.NonCartOp(maps, psi, traj, normal_mode="gridding")
