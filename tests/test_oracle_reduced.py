"""Pins of the reduced-resolution grid oracle (oracle/reduced.py)."""
import numpy as np

import workloads
from oracle import nufft as onufft
from oracle import pico as opico
from oracle import reduced, sense


def test_uniform_undersampling_coarse_variance_equals_native_at_coarse_pixels():
    """For uniform R without calibration lines the native variance at a pixel
    depends only on the maps at that pixel and its R - 1 aliases ny/R apart
    (closed-form SENSE); the coarse problem aliases the same native pixels,
    so its exact variance equals the native closed form at pixels f m.  A
    wrong map sampling, mask block or centre alignment breaks the equality."""
    rng = np.random.default_rng(1)
    maps = workloads.coil_maps(64, 48, 4, rng)
    psi = workloads.noise_cov(4, rng)
    mask = workloads.cart_mask_1d(64, 2, 0)
    var_native, _, _ = sense.sense_closed_form(maps, psi, 2)
    for f in (2, 4):
        cm, ck = reduced.coarse_maps(maps, f), reduced.coarse_mask(mask, f)
        assert ck.sum() == ck.size // 2
        op = opico.cartesian(cm, psi, ck)
        var_coarse = sense.exact_diag_1d(op, ck)
        err = np.abs(var_coarse - var_native[::f, ::f]).max() / var_native.max()
        assert err < 1e-12


def test_full_sampling_keeps_variance_level():
    """Fully sampled: native and coarse variances are both 1 / sum_c |S_w,c|^2."""
    rng = np.random.default_rng(2)
    maps = workloads.coil_maps(32, 32, 3, rng)
    mask = np.ones(32, np.uint8)
    op = opico.cartesian(reduced.coarse_maps(maps, 2), None, reduced.coarse_mask(mask, 2))
    v = sense.exact_diag_1d(op, reduced.coarse_mask(mask, 2))
    ref = 1.0 / np.sum(np.abs(maps[:, ::2, ::2]) ** 2, axis=0)
    assert np.abs(v - ref).max() < 1e-12 * ref.max()


def test_coarse_mask_and_traj_selection():
    m2 = np.arange(64 * 32).reshape(64, 32) % 7
    c = reduced.coarse_mask(m2, 4)
    assert c.shape == (16, 8) and np.array_equal(c, m2[24:40, 12:20])
    t = np.array([[0.0, 0.0], [np.pi / 2 - 1e-9, -np.pi / 2], [np.pi / 2, 0.0], [-3.0, 0.1], [0.3, -0.2]])
    ct = reduced.coarse_traj(t, 2)
    assert np.allclose(ct, np.array([[0.0, 0.0], [np.pi - 2e-9, -np.pi], [0.6, -0.4]]))


def test_noncart_coarse_operator_is_the_band_limited_acquisition():
    """A coarse image placed on native pixels f m (zeros elsewhere) gives the
    same NUDFT data on the kept samples as the coarse image on the coarse
    grid: the scaled trajectory and the centre alignment agree."""
    rng = np.random.default_rng(3)
    traj = rng.uniform(-np.pi, np.pi, (400, 2))
    ct = reduced.coarse_traj(traj, 2)
    keep = np.all((traj >= -np.pi / 2) & (traj < np.pi / 2), axis=1)
    xc = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    xn = np.zeros((16, 16), complex)
    xn[::2, ::2] = xc
    a = onufft.nudft_forward(xn, traj[keep]) * np.sqrt(16 * 16)
    b = onufft.nudft_forward(xc, ct) * np.sqrt(8 * 8)
    assert np.abs(a - b).max() < 1e-10 * np.abs(b).max()


def test_bilinear_upsampling():
    rng = np.random.default_rng(4)
    c = rng.random((6, 5))
    u = reduced.upsample_bilinear(c, 4)
    assert u.shape == (24, 20)
    assert np.array_equal(u[::4, ::4], c)                      # nodes kept
    assert np.allclose(u[2, 0], 0.5 * (c[0, 0] + c[1, 0]))     # midpoints
    assert np.allclose(u[0, 18], 0.5 * (c[0, 4] + c[0, 0]))    # periodic wrap
    assert np.allclose(reduced.upsample_bilinear(np.full((3, 3), 2.5), 2), 2.5)
    # separable linear ramp inside the period is reproduced exactly
    ramp = np.add.outer(np.arange(6) * 1.0, np.arange(5) * 2.0)
    assert np.allclose(reduced.upsample_bilinear(ramp, 2)[:10, :8],
                       np.add.outer(np.arange(10) * 0.5, np.arange(8) * 1.0))
