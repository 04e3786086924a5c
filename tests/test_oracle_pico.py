"""Pins of the oracle's PICO estimator, Tikhonov composition and PMR.

  * Exact enumeration over every QPSK / Rademacher probe on tiny grids makes
    the estimator exactly diag(Sigma) (unbiasedness, Sec. 2.2, Eq. (16)),
    with Sigma from a dense LAPACK inverse.
  * The enumerated per-voxel variance equals the Re-part of App. B, Eq. (A1):
    1/2 sum_{l!=k} |Sigma_kl|^2 (random phase / QPSK, kappa = 1) and
    sum_{l!=k} (Re Sigma_kl)^2 (real Rademacher).
  * Full sampling (Sigma diagonal): a single random-phase probe is exact.
  * Tikhonov: the two-solve composition equals (M+l)^-1 M (M+l)^-1 and its
    diagonal lies below diag(M^-1) (App. D, Proposition).
  * PMR converges to diag(Sigma) at the 1/sqrt(N) rate (App. C).
  * Continuous random phase: z-scores of the estimate are standard (CLT).
"""
import itertools

import numpy as np
import pytest

import workloads
from oracle import pico, sense


def _op(ny, nx, nc=2, R=2, acs=0, seed=1, full=False):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(ny, nx, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    mask = np.ones(ny, np.uint8) if full else workloads.cart_mask_1d(ny, R, acs)
    return pico.cartesian(maps, psi, mask)


def _enum(values, n, shape):
    for combo in itertools.product(values, repeat=n):
        yield np.array(combo, np.complex128).reshape(shape)


def test_qpsk_enumeration_is_exact_and_matches_A1():
    op = _op(4, 1, nc=2)
    cov = pico.Covariance(op, 0.0, cg_iters=12)
    Sigma = np.linalg.inv(op.dense_normal())
    acc = pico.noise_map(cov, 0, 0, 0, probes=_enum([1, 1j, -1, -1j], 4, (4, 1)))
    assert acc["count"] == 256
    est = pico.finalize(acc).ravel()
    assert np.allclose(est, np.real(np.diag(Sigma)), rtol=1e-10, atol=0)
    assert np.abs(acc["sum_im"] / acc["count"]).max() < 1e-9 * est.max()
    var = acc["sumsq"].ravel() / acc["count"] - est ** 2
    off = np.abs(Sigma) ** 2
    np.fill_diagonal(off, 0)
    assert np.allclose(var, 0.5 * off.sum(1), rtol=1e-8)


def test_rademacher_enumeration_is_exact_and_matches_re_part_variance():
    op = _op(4, 2, nc=2)
    cov = pico.Covariance(op, 0.0, cg_iters=16)
    Sigma = np.linalg.inv(op.dense_normal())
    acc = pico.noise_map(cov, 0, 0, 0, probes=_enum([1, -1], 8, (4, 2)))
    est = pico.finalize(acc).ravel()
    assert np.allclose(est, np.real(np.diag(Sigma)), rtol=1e-9, atol=0)
    var = acc["sumsq"].ravel() / acc["count"] - est ** 2
    off = np.real(Sigma) ** 2
    np.fill_diagonal(off, 0)
    assert np.allclose(var, off.sum(1), rtol=1e-7)


def test_tikhonov_composition_enumeration_and_shrinkage():
    op = _op(4, 1, nc=2)
    cov = pico.Covariance(op, 0.3, cg_iters=12)
    assert cov.lam > 0
    Md = op.dense_normal()
    Ri = np.linalg.inv(Md + cov.lam * np.eye(4))
    Sig_l = Ri @ Md @ Ri
    acc = pico.noise_map(cov, 0, 0, 0, probes=_enum([1, 1j, -1, -1j], 4, (4, 1)))
    assert np.allclose(pico.finalize(acc).ravel(), np.real(np.diag(Sig_l)), rtol=1e-9)
    # App. D: Sigma_lam < Sigma_LS in the Loewner order, so the diagonal shrinks
    Sig_ls = np.linalg.inv(Md)
    assert np.linalg.eigvalsh(Sig_ls - Sig_l).min() > 0
    big = _op(16, 8, nc=3, acs=2)
    d_ls = sense.exact_diag_1d(big, big.P[:, 0])
    d_l = sense.exact_diag_1d(big, big.P[:, 0], lam=0.05)
    assert np.all(d_l < d_ls)


def test_full_sampling_single_probe_exact():
    op = _op(4, 2, nc=2, full=True)
    cov = pico.Covariance(op, 0.0, cg_iters=16)
    acc = pico.noise_map(cov, 9, 0, 1)
    Sw = sense.whiten_maps(*_maps_psi(4, 2, 2, 1))
    exact = 1.0 / np.sum(np.abs(Sw) ** 2, axis=0)
    assert np.allclose(pico.finalize(acc), exact, rtol=1e-10)
    # a complex Gaussian probe (kappa = 2) is not exact with one sample
    acc_g = pico.noise_map(cov, 9, 0, 1, dist="gaussian")
    assert np.abs(pico.finalize(acc_g) / exact - 1).max() > 0.05


def _maps_psi(ny, nx, nc, seed):
    rng = np.random.default_rng(seed)
    return workloads.coil_maps(ny, nx, nc, rng), workloads.noise_cov(nc, rng)


def test_random_phase_z_scores_are_standard():
    op = _op(16, 8, nc=3, R=2)
    Sigma = np.linalg.inv(op.dense_normal())
    N = 300
    cov = pico.Covariance(op, 0.0, cg_iters=60)
    acc = pico.noise_map(cov, 21, 0, N)
    est = pico.finalize(acc).ravel()
    off = np.abs(Sigma) ** 2
    np.fill_diagonal(off, 0)
    z = (est - np.real(np.diag(Sigma))) / np.sqrt(0.5 * off.sum(1) / N)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert 0.7 < z.var() < 1.3


def test_resume_split_equals_single_call():
    op = _op(8, 4, nc=2)
    cov = pico.Covariance(op, 0.0, cg_iters=10)
    a = pico.noise_map(cov, 4, 0, 6)
    b = pico.noise_map(cov, 4, 0, 2)
    b = pico.noise_map(cov, 4, 2, 4, acc=b)
    assert np.array_equal(a["sum"], b["sum"]) and a["count"] == b["count"]


def test_pmr_converges_to_exact_diagonal():
    op = _op(8, 4, nc=2, R=2, acs=2)
    exact = sense.exact_diag_1d(op, op.P[:, 0])
    cov = pico.Covariance(op, 0.0, cg_iters=40)
    N = 1500
    acc = pico.pmr(cov, 17, 0, N)
    var = pico.pmr_finalize(acc)
    rel = var / exact
    assert abs(rel.mean() - 1) < 4 / np.sqrt(N * rel.size)
    assert pico.nrmse_var(var, exact) < 2.5 / np.sqrt(N)


def test_pmr_hybrid_noise_is_white_on_the_mask():
    op = _op(16, 8, nc=2, R=2, acs=2)
    n = np.stack([pico.pmr_noise(op, 3, r) for r in range(200)])
    on = op.P[None, None] > 0
    p = np.mean(np.abs(n) ** 2, axis=0)
    assert np.all(n[:, :, op.P == 0] == 0)
    assert abs(p[np.broadcast_to(on[0], p.shape)].mean() - 1) < 0.03


def test_nrmse_and_certify():
    ref = np.full((4, 4), 4.0)
    assert pico.nrmse_std(ref * 1.0201, ref) == pytest.approx(0.01, rel=1e-6)
    maps = {100: ref * 1.05, 200: ref * 1.04, 400: ref * 1.001, 800: ref * 1.0005}
    assert pico.certify(maps, ref) == 400


def test_exact_columns_estimator_matches_converged_cg():
    op = _op(16, 6, nc=3, R=2, acs=2)
    cov = pico.Covariance(op, 0.0, cg_iters=80)
    acc = pico.noise_map(cov, 5, 0, 3)
    cols = [0, 3, 5]
    ex = pico.noise_map_exact_columns(op, op.P[:, 0], 5, 0, 3, cols)
    assert np.allclose(acc["sum"][:, cols], ex, rtol=1e-9, atol=1e-12)
    cov_l = pico.Covariance(op, 0.2, cg_iters=80)
    acc_l = pico.noise_map(cov_l, 5, 0, 3)
    ex_l = pico.noise_map_exact_columns(op, op.P[:, 0], 5, 0, 3, cols, lam=cov_l.lam)
    assert np.allclose(acc_l["sum"][:, cols], ex_l, rtol=1e-9, atol=1e-12)


def test_stderr_proxy_matches_closed_form_and_monte_carlo():
    # per-voxel variance of the random-phase terms: E[s2_k] = 1/2 sum_{l!=k} |Sigma_kl|^2
    # (Re part of App. B, Eq. (A1)); and the proxy predicts the RMS std-map NRMSE
    # of independent N-probe runs against the exact diagonal
    op = _op(16, 8, nc=3, R=2)
    Sigma = np.linalg.inv(op.dense_normal())
    off = np.abs(Sigma) ** 2
    np.fill_diagonal(off, 0)
    half = 0.5 * off.sum(1)
    exact = np.real(np.diag(Sigma))
    cov = pico.Covariance(op, 0.0, cg_iters=60)
    big = pico.noise_map(cov, 3, 0, 2000)
    N = big["count"]
    m = big["sum"].ravel() / N
    s2 = (big["sumsq"].ravel() - N * m * m) / (N - 1)
    assert abs(s2.mean() / half.mean() - 1.0) < 0.06
    errs, proxies = [], []
    for r in range(40):
        acc = pico.noise_map(cov, 5, 24 * r, 24)
        errs.append(pico.nrmse_std(pico.finalize(acc), exact.reshape(acc["sum"].shape)))
        proxies.append(pico.stderr_proxy(acc))
    rms = float(np.sqrt(np.mean(np.square(errs))))
    assert abs(np.mean(proxies) / rms - 1.0) < 0.2
    # a diagonal covariance (full sampling, one coil of unit magnitude) makes
    # every probe exact: zero spread, zero proxy
    yy, xx = np.meshgrid(np.arange(8), np.arange(4), indexing="ij")
    maps = np.exp(2j * np.pi * 0.1 * yy)[None] * np.ones((1, 8, 4))
    op1 = pico.cartesian(maps, np.array([[2.0]]), np.ones(8, np.uint8))
    acc = pico.noise_map(pico.Covariance(op1, 0.0, cg_iters=4), 1, 0, 5)
    assert pico.stderr_proxy(acc) < 1e-7          # rounding of sumsq - N m^2 only


def test_bf16_rounding_matches_library_conversion():
    """oracle.storage rounds like torch's CPU float32 -> bfloat16 conversion
    (round to nearest, ties to even), including exact ties, signed zeros,
    infinities and values next to the largest finite bfloat16."""
    import torch
    from oracle import storage
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
        # exact ties: low 16 bits 0x8000 over odd and even kept halves
        (np.arange(0x3F800000, 0x3F800000 + 64 * 0x10000, 0x10000, dtype=np.uint32) + 0x8000).view(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, -3.3895314e38, 1e-40], np.float32),
    ])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = storage.bf16_round_real(x)
    assert np.array_equal(got, ref)
    assert np.isnan(storage.bf16_round_real(np.array([np.nan], np.float32))[0])
    # relative rounding error is at most the unit roundoff 2^-8 (8 significant bits)
    ok = np.isfinite(ref) & (np.abs(x) > 1e-30)
    assert np.max(np.abs(got[ok] - x[ok]) / np.abs(x[ok])) <= 2.0 ** -8
    z = (rng.standard_normal(50) + 1j * rng.standard_normal(50)).astype(np.complex64)
    zq = storage.bf16_round(z)
    assert np.array_equal(zq.real, storage.bf16_round_real(z.real))
    assert np.array_equal(zq.imag, storage.bf16_round_real(z.imag))
