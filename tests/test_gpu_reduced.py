"""Reduced-resolution noise grid on the GPU (pico_init_reduced /
pico_upsample_map) against the oracle's statement of the coarse problem and
of the interpolation (oracle/reduced.py), and its accuracy against the
native exact map."""
import sys

import numpy as np
import pytest

import workloads
from oracle import nufft as onufft
from oracle import pico as opico
from oracle import reduced

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2605_09590_amd import pico as lib
    lib.load()
    assert torch.cuda.is_available()
    return lib


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _map(lib, h, n, seed, nprobes):
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    acc = lib.make_accum(acc_t[0], None, acc_t[1])
    lib.pico_noise_map(h, seed, 0, nprobes, 0, acc)
    var = torch.empty(n, dtype=torch.float64, device="cuda:0")
    lib.pico_finalize(h, acc, var)
    torch.cuda.synchronize()
    return var


def test_reduced_phase_encode_parity_and_upsampling(lib):
    say("case: phase-encode native 128x96, 4 coils, R=2 + 8 ACS, factor 2 (coarse 64x48), 12 probes in "
        "tiles of 8, CG 20; coarse map vs the oracle's coarse problem, upsampled map vs its interpolation")
    rng = np.random.default_rng(5)
    maps = workloads.coil_maps(128, 96, 4, rng)
    psi = workloads.noise_cov(4, rng)
    mask = workloads.cart_mask_1d(128, 2, 8)
    h = lib.pico_init_reduced(2, 128, 96, _dev(maps.astype(np.complex64)), psi, _dev(mask), cg_iters=20,
                              probe_tile=8)
    var_c = _map(lib, h, 64 * 48, 3, 12)
    up = torch.empty(128 * 96, dtype=torch.float64, device="cuda:0")
    lib.pico_upsample_map(h, var_c, up)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cm = reduced.coarse_maps(maps.astype(np.complex64).astype(np.complex128), 2)
    ref = opico.noise_map(opico.Covariance(opico.cartesian(cm, psi, reduced.coarse_mask(mask, 2)), 0.0, 20), 3, 0, 12)
    e = _rel(var_c.cpu().numpy(), opico.finalize(ref).ravel())
    say(f"  coarse map rel err {e:.2e}")
    assert e < TOL
    eu = _rel(up.cpu().numpy(), reduced.upsample_bilinear(var_c.cpu().numpy().reshape(64, 48), 2).ravel())
    say(f"  upsampled map vs oracle interpolation of the same coarse map {eu:.2e}")
    assert eu < 1e-13


def test_reduced_cart2d_apply_cov(lib):
    say("case: Cartesian 2-D Poisson-disc native 128x128, 5 coils, lambda 0.05, factor 2 (coarse 64x64), "
        "apply_cov on 2 probes, CG 20")
    rng = np.random.default_rng(6)
    maps = workloads.coil_maps(128, 128, 5, rng)
    psi = workloads.noise_cov(5, rng)
    mask = workloads.poisson_disc_mask(128, 128, 2.0, 16, seed=2)
    h = lib.pico_init_reduced(2, 128, 128, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                              sampling=lib.PICO_CART_2D, lam=0.05, cg_iters=20, probe_tile=2)
    v = rng.standard_normal((2, 64, 64)) + 1j * rng.standard_normal((2, 64, 64))
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 2)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cm = reduced.coarse_maps(maps.astype(np.complex64).astype(np.complex128), 2)
    cov = opico.Covariance(opico.cartesian(cm, psi, reduced.coarse_mask(mask, 2)), 0.05, 20)
    for k in range(2):
        e = _rel(ut.cpu().numpy()[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL


def test_reduced_spiral_noise_map(lib):
    say("case: spiral native 128x128, 4 coils, 24x2048 R=1, lambda 0.1, factor 2 (coarse 64x64, Toeplitz "
        "grid 128), 8 probes in tiles of 4, CG 20")
    rng = np.random.default_rng(7)
    maps = workloads.coil_maps(128, 128, 4, rng)
    psi = workloads.noise_cov(4, rng)
    traj = workloads.spiral_traj(128, 1, 24, 2048).astype(np.float32)
    h = lib.pico_init_reduced(2, 128, 128, _dev(maps.astype(np.complex64)), psi, None,
                              sampling=lib.PICO_NONCART, lam=0.1, cg_iters=20, probe_tile=4, traj=_dev(traj),
                              nsamples=traj.shape[0])
    var_c = _map(lib, h, 64 * 64, 9, 8)
    lib.pico_destroy(h)
    ct = reduced.coarse_traj(traj.astype(np.float64), 2).astype(np.float32).astype(np.float64)
    say(f"  {ct.shape[0]} of {traj.shape[0]} samples in the coarse band")
    cm = reduced.coarse_maps(maps.astype(np.complex64).astype(np.complex128), 2)
    ref = opico.noise_map(opico.Covariance(onufft.NonCartOp(cm, psi, ct), 0.1, 20), 9, 0, 8)
    e = _rel(var_c.cpu().numpy(), opico.finalize(ref).ravel())
    say(f"  coarse map rel err {e:.2e}")
    assert e < TOL


def test_reduced_argument_errors(lib):
    say("case: reduced-grid argument errors (factor, divisibility, CS, upsampling a native operator)")
    rng = np.random.default_rng(8)
    maps = _dev(workloads.coil_maps(128, 96, 2, rng).astype(np.complex64))
    mask = _dev(workloads.cart_mask_1d(128, 2, 8))
    for f in (1, 3, 5):
        with pytest.raises(lib.PicoError) as ei:
            lib.pico_init_reduced(f, 128, 96, maps, None, mask, cg_iters=5, probe_tile=2)
        assert ei.value.status == lib.PICO_EINVAL
    m2 = _dev(np.ones((128, 96), np.uint8))
    with pytest.raises(lib.PicoError) as ei:
        lib.pico_init_reduced(2, 128, 96, maps, None, m2, sampling=lib.PICO_CART_2D,
                              recon=lib.PICO_CS_FISTA_L1WAV, kdata=maps, fista_iters=5)
    assert ei.value.status == lib.PICO_EUNSUPPORTED
    h = lib.pico_init(128, 96, maps, None, mask, cg_iters=5, probe_tile=2)
    x = torch.zeros(128 * 96, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lib.PicoError) as ei:
        lib.pico_upsample_map(h, x, x)
    assert ei.value.status == lib.PICO_EUNSUPPORTED
    lib.pico_destroy(h)


def test_reduced_grid_accuracy_full_size(lib):
    say("case: accuracy of the reduced grid at 320x320, 15 coils, R=2 + 24 ACS: exact coarse maps "
        "(factor 2: 160x160) upsampled vs the native exact map")
    prob = workloads.config(2, seed=0)
    maps = _dev(prob.maps.astype(np.complex64))
    mask = _dev(prob.mask)
    h = lib.pico_init(320, 320, maps, prob.psi, mask, cg_iters=60, probe_tile=64)
    ref = torch.empty(320 * 320, dtype=torch.float64, device="cuda:0")
    lib.pico_exact_diag(h, ref)
    lib.pico_destroy(h)
    hc = lib.pico_init_reduced(2, 320, 320, maps, prob.psi, mask, cg_iters=60, probe_tile=64)
    vc = torch.empty(160 * 160, dtype=torch.float64, device="cuda:0")
    lib.pico_exact_diag(hc, vc)
    up = torch.empty_like(ref)
    lib.pico_upsample_map(hc, vc, up)
    torch.cuda.synchronize()
    lib.pico_destroy(hc)
    s, s0 = torch.sqrt(torch.clamp(up, min=0)), torch.sqrt(torch.clamp(ref, min=0))
    e = float(torch.linalg.norm(s - s0) / torch.linalg.norm(s0))
    at_nodes = float(torch.linalg.norm((s - s0).reshape(320, 320)[::2, ::2]) / torch.linalg.norm(s0.reshape(320, 320)[::2, ::2]))
    say(f"  std-map NRMSE of the upsampled exact coarse map {e:.4f} (at the coarse pixels {at_nodes:.4f})")
    assert e < 0.05
