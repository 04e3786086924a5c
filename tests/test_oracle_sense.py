"""Pins of the oracle's whitened Cartesian SENSE operators (Sec. 2.1).

Closed forms and brute force, none of which reuse the code under test:
  * classical SENSE unfolding with the noise covariance (no whitening code),
  * dense inverse built column by column from the FFT operators,
  * full sampling makes M diagonal with entries sum_c |s_w,c|^2,
  * adjointness <A x, y> = <x, A^H y>.
"""
import numpy as np
import pytest

import workloads
from oracle import pico, sense


def _tiny(ny=8, nx=4, nc=3, R=2, acs=0, seed=1):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(ny, nx, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    mask = workloads.cart_mask_1d(ny, R, acs)
    return maps, psi, mask


def test_closed_form_matches_unwhitened_sense_formula():
    # var_acc = R [(S^H Psi^-1 S)^-1]_mm : Pruessmann's SENSE noise formula,
    # evaluated directly from the raw maps and Psi (no Cholesky, no FFT).
    p = workloads.config(1, seed=0)
    va, vr, g = sense.sense_closed_form(p.maps, p.psi, 2)
    Pi = np.linalg.inv(p.psi)
    ny = p.ny
    for x in (0, 17, 40, 63):
        for y0 in (0, 5, 31):
            ys = [y0, y0 + ny // 2]
            S = p.maps[:, ys, x]
            G = S.conj().T @ Pi @ S
            Gi = np.linalg.inv(G)
            for m, y in enumerate(ys):
                assert va[y, x] == pytest.approx(2 * Gi[m, m].real, rel=1e-12)
                assert vr[y, x] == pytest.approx(1 / G[m, m].real, rel=1e-12)
    assert g.min() >= 1.0 - 1e-12          # unregularised SENSE: g >= 1


def test_closed_form_equals_dense_columnwise_inverse_config1():
    p = workloads.config(1, seed=0)
    op = pico.cartesian(p.maps, p.psi, p.mask)
    va, _, _ = sense.sense_closed_form(p.maps, p.psi, 2)
    ex = sense.exact_diag_1d(op, p.mask)
    assert np.max(np.abs(va - ex) / ex) < 1e-12


@pytest.mark.parametrize("acs", [0, 4])
def test_columnwise_blocks_equal_full_dense_inverse(acs):
    maps, psi, mask = _tiny(ny=8, nx=4, acs=acs)
    op = pico.cartesian(maps, psi, mask)
    full = np.linalg.inv(op.dense_normal())
    blk = sense.exact_diag_1d(op, mask)
    assert np.allclose(np.real(np.diag(full)).reshape(8, 4), blk, rtol=1e-11, atol=0)
    # and M really is block diagonal over image columns for a 1-D mask
    Md = op.dense_normal().reshape(8, 4, 8, 4)
    off = sum(np.abs(Md[:, a, :, b]).max() for a in range(4) for b in range(4) if a != b)
    assert off < 1e-13


def test_full_sampling_gives_diagonal_normal_operator():
    maps, psi, _ = _tiny(ny=8, nx=4)
    op = pico.cartesian(maps, psi, np.ones(8, np.uint8))
    Md = op.dense_normal()
    Sw = sense.whiten_maps(maps, psi)
    d = np.sum(np.abs(Sw) ** 2, axis=0).ravel()
    assert np.allclose(Md, np.diag(d), atol=1e-13)


def test_adjoint_and_hermitian():
    maps, psi, mask = _tiny(ny=16, nx=8, acs=2)
    for m in (mask, workloads.cart_mask_2d_uniform(16, 8, 2, 2)):
        op = pico.cartesian(maps, psi, m)
        rng = np.random.default_rng(4)
        x = rng.standard_normal((16, 8)) + 1j * rng.standard_normal((16, 8))
        y = rng.standard_normal((3, 16, 8)) + 1j * rng.standard_normal((3, 16, 8))
        lhs = np.vdot(op.forward(x), y)
        rhs = np.vdot(x, op.adjoint(y))
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        Md = op.dense_normal()
        assert np.allclose(Md, Md.conj().T, atol=1e-13)
        assert np.linalg.eigvalsh(Md).min() > -1e-12


def test_noise_covariance_scaling():
    # Psi -> c Psi scales every voxel variance by c (whitening is linear in L)
    maps, psi, mask = _tiny()
    op1 = pico.cartesian(maps, psi, mask)
    op2 = pico.cartesian(maps, 3.0 * psi, mask)
    d1 = sense.exact_diag_1d(op1, mask)
    d2 = sense.exact_diag_1d(op2, mask)
    assert np.allclose(d2, 3.0 * d1, rtol=1e-12)


def test_whitening_identity_when_psi_is_identity():
    maps, _, _ = _tiny()
    assert np.array_equal(sense.whiten_maps(maps, None), maps)
    assert np.allclose(sense.whiten_maps(maps, np.eye(3)), maps, atol=0)
