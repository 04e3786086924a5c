"""Pins of the oracle's CG and power method against LAPACK."""
import numpy as np

import workloads
from oracle import pico, solvers


def _op(ny=16, nx=16, nc=3, seed=2, acs=0):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(ny, nx, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    return pico.cartesian(maps, psi, workloads.cart_mask_1d(ny, 2, acs))


def test_converged_cg_equals_dense_solve():
    op = _op()
    Md = op.dense_normal()
    b = pico.probe_image(3, 0, (16, 16))
    for lam in (0.0, 0.7):
        x = solvers.cg(op.normal, b, 200, lam=lam)
        ref = np.linalg.solve(Md + lam * np.eye(256), b.ravel())
        assert np.linalg.norm(x.ravel() - ref) < 1e-9 * np.linalg.norm(ref)


def test_cg_tolerance_mode_stops_at_tol():
    op = _op()
    b = pico.probe_image(3, 1, (16, 16))
    x, info = solvers.cg(op.normal, b, 500, tol=1e-3, return_info=True)
    assert info["relres"] <= 1e-3
    assert info["iters"] < 500
    r = b - op.normal(x)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-3


def test_cg_breakdown_freezes():
    b = np.ones((4, 4), np.complex128)
    x, info = solvers.cg(lambda p: -p, b, 10, return_info=True)
    assert info["frozen"] and np.all(x == 0)


def test_power_method_on_known_spectrum():
    # diagonal operator with a clear spectral gap: the Rayleigh quotient
    # converges like (l2/l1)^(2k) to l1
    d = np.linspace(0.1, 1.0, 64).reshape(8, 8)
    d[3, 4] = 2.0
    est = solvers.power_method(lambda v: d * v, (8, 8), iters=40, margin=1.0)
    assert abs(est - 2.0) < 1e-10
    assert solvers.power_method(lambda v: d * v, (8, 8), iters=40) == 1.01 * est


def test_power_method_bounded_and_monotone_on_sense():
    op = _op()
    lmax = np.linalg.eigvalsh(op.dense_normal()).max()
    prev = 0.0
    for it in (1, 5, 15, 60):
        est = solvers.power_method(op.normal, (16, 16), iters=it, margin=1.0)
        assert prev - 1e-12 <= est <= lmax * (1 + 1e-12)   # Rayleigh quotients rise to lmax
        prev = est
    assert prev > 0.95 * lmax
