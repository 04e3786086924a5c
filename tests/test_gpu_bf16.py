"""bfloat16 storage (pico_storage_t) on the GPU against the FP64 oracle.

Two comparisons per case:
* against the oracle operator built from the same bfloat16-rounded whitened
  maps (oracle.storage): the rounding of the maps is then part of the
  operator on both sides, and the GPU must agree to the FP32 bar (1e-4);
* against the unrounded operator: the total effect of bfloat16 storage,
  bar 1e-2.
With PICO_BF16_STREAM the grid path also keeps its row-transformed coil
planes in bfloat16; that rounding sits inside the operator and only the
1e-2 bar applies.  For the nonlinear CS map bfloat16 is a storage form of
the tangents' normal-operator reads only: the FP64 primal (the linearisation
point, whose active set fixes the Jacobian) and the k-space adjoint of the
probes use the unrounded maps, so the reconstruction meets the FP32 bar
against the FP64-map oracle and the Jacobian probes and their noise map the
1e-2 bar; at full size the bfloat16 noise map is compared with the FP32-storage
map of the same probes.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import cs as ocs
from oracle import nufft as onufft
from oracle import pico as opico
from oracle import storage as ostore

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_BF16 = 1e-2


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


def _gpu_map(lib, h, n, seed, first, nprobes):
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lib.pico_noise_map(h, seed, first, nprobes, 0, lib.make_accum(*acc_t))
    torch.cuda.synchronize()
    return acc_t[0].cpu().numpy()


@pytest.mark.parametrize("form", [0, 2, 3])
def test_bf16_maps_phase_encode(lib, form):
    say(f"case: phase-encode 64x64, 4 coils, R=2, 16 probes in tiles of 8, CG 20, bfloat16 maps, "
        f"normal form {form} (the dense blocks are built from the rounded maps)")
    prob = workloads.config(1, seed=0)
    h = lib.pico_init(64, 64, _dev(prob.maps.astype(np.complex64)), prob.psi, _dev(prob.mask),
                      cg_iters=20, probe_tile=8, storage=lib.PICO_BF16_MAPS, normal_form=form)
    s = _gpu_map(lib, h, 64 * 64, 4, 0, 16)
    lib.pico_destroy(h)
    wq = ostore.bf16_whitened_maps(prob.maps, prob.psi)
    ref_q = opico.noise_map(opico.Covariance(opico.cartesian(wq, None, prob.mask), 0.0, 20), 4, 0, 16)
    ref = opico.noise_map(opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 20), 4, 0, 16)
    eq, e = _rel(s, ref_q["sum"].ravel()), _rel(s, ref["sum"].ravel())
    say(f"  vs rounded-map oracle {eq:.2e}; vs FP64 maps {e:.2e}")
    assert eq < TOL and e < TOL_BF16


# bfloat16 maps on the FFT path for the column plans of every family: two-step
# plans with the mask weights in registers (160, 288) or selected from the
# mask bits (384: 24-lane groups), and the 64-lane Stockham plan (512)
@pytest.mark.parametrize("ny,nx,nc", [(160, 24, 4), (288, 16, 3), (384, 12, 3), (512, 8, 2)])
def test_bf16_maps_fft_form_column_lengths(lib, ny, nx, nc):
    say(f"case: phase-encode {ny}x{nx}, {nc} coils, R=2 + 8 ACS, 9 probes in tiles of 5, CG 20, "
        f"bfloat16 maps, FFT form")
    prob = workloads.config(2, seed=ny + 3, ny=ny, nx=nx, nc=nc, acs=8, cg_iters=20)
    h = lib.pico_init(ny, nx, _dev(prob.maps.astype(np.complex64)), prob.psi, _dev(prob.mask),
                      cg_iters=20, probe_tile=5, storage=lib.PICO_BF16_MAPS, normal_form=0)
    s = _gpu_map(lib, h, ny * nx, 6, 0, 9)
    lib.pico_destroy(h)
    wq = ostore.bf16_whitened_maps(prob.maps, prob.psi)
    ref_q = opico.noise_map(opico.Covariance(opico.cartesian(wq, None, prob.mask), 0.0, 20), 6, 0, 9)
    eq = _rel(s, ref_q["sum"].ravel())
    say(f"  vs rounded-map oracle {eq:.2e}")
    assert eq < TOL


@pytest.mark.parametrize("storage", [1, 2])
def test_bf16_cart2d_apply_cov(lib, storage):
    say(f"case: Cartesian 2-D Poisson-disc 64x96, 5 coils, lambda 0.05, apply_cov on 3 probes, CG 20, "
        f"storage {storage}")
    rng = np.random.default_rng(12)
    maps = workloads.coil_maps(64, 96, 5, rng)
    psi = workloads.noise_cov(5, rng)
    mask = workloads.poisson_disc_mask(64, 96, 2.0, 12, seed=4)
    h = lib.pico_init(64, 96, _dev(maps.astype(np.complex64)), psi, _dev(mask), sampling=lib.PICO_CART_2D,
                      lam=0.05, cg_iters=20, probe_tile=4, storage=storage)
    v = rng.standard_normal((3, 64, 96)) + 1j * rng.standard_normal((3, 64, 96))
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 3)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    u = ut.cpu().numpy()
    cov_q = opico.Covariance(opico.cartesian(ostore.bf16_whitened_maps(maps, psi), None, mask), 0.05, 20)
    cov = opico.Covariance(opico.cartesian(maps, psi, mask), 0.05, 20)
    for k in range(3):
        eq, e = _rel(u[k], cov_q.apply(v[k])), _rel(u[k], cov.apply(v[k]))
        say(f"  probe {k}: vs rounded-map oracle {eq:.2e}; vs FP64 maps {e:.2e}")
        assert e < TOL_BF16
        if storage == 1:
            assert eq < TOL


@pytest.mark.parametrize("storage", [1, 2])
def test_bf16_spiral_noise_map(lib, storage):
    say(f"case: spiral Toeplitz 64x64, 4 coils, 16x512 R=2, lambda 0.1, 8 probes in tiles of 4, CG 20, "
        f"storage {storage}")
    rng = np.random.default_rng(3)
    maps = workloads.coil_maps(64, 64, 4, rng)
    psi = workloads.noise_cov(4, rng)
    traj = workloads.spiral_traj(64, 2, 16, 512).astype(np.float32)
    h = lib.pico_init(64, 64, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART,
                      lam=0.1, cg_iters=20, probe_tile=4, traj=_dev(traj), nsamples=traj.shape[0],
                      storage=storage)
    s = _gpu_map(lib, h, 64 * 64, 9, 0, 8)
    lib.pico_destroy(h)
    t64 = traj.astype(np.float64)
    ref_q = opico.noise_map(opico.Covariance(onufft.NonCartOp(ostore.bf16_whitened_maps(maps, psi), None, t64),
                                             0.1, 20), 9, 0, 8)
    ref = opico.noise_map(opico.Covariance(onufft.NonCartOp(maps, psi, t64), 0.1, 20), 9, 0, 8)
    eq, e = _rel(s, ref_q["sum"].ravel()), _rel(s, ref["sum"].ravel())
    say(f"  vs rounded-map oracle {eq:.2e}; vs FP64 maps {e:.2e}")
    assert e < TOL_BF16
    if storage == 1:
        assert eq < TOL


def _std_nrmse(a, b):
    sa, sb = np.sqrt(np.maximum(a, 0)), np.sqrt(np.maximum(b, 0))
    return float(np.linalg.norm(sa - sb) / np.linalg.norm(sb))


def _cs_case(n_y, n_x, nc, seed, calib=8):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n_y, n_x, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    x = workloads.phantom(max(n_y, n_x), rng)[:n_y, :n_x]
    mask = workloads.poisson_disc_mask(n_y, n_x, 2.0, calib, seed=seed)
    op = opico.cartesian(maps, psi, mask)
    bw = op.forward(x)
    bw = bw + 1e-3 * op.P[None] * (rng.standard_normal(bw.shape) + 1j * rng.standard_normal(bw.shape))
    braw = np.einsum("cd,dyx->cyx", np.linalg.cholesky(psi), bw)
    return maps, psi, mask, op, bw, braw


def _cs_check(lib, h, f, op, bw, shape, nprobe_map=6):
    """Reconstruction (FP32 bar), 2 Jacobian probes and a 6-probe |J w|^2 map
    (1e-2 bar) against the FP64-map oracle ``f``."""
    ny, nx = shape
    w = np.stack([ocs.kspace_probe(op, 8, i) for i in range(2)])
    ut = torch.empty((2, ny, nx), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_jvp(h, _dev(w.astype(np.complex64)), ut, 2)
    xg = torch.empty((ny, nx), dtype=torch.complex64, device="cuda:0")
    lib.pico_recon(h, xg)
    g = _gpu_map(lib, h, ny * nx, 21, 0, nprobe_map)
    torch.cuda.synchronize()
    xr, cr = f.recon(bw, store=True)
    e = _rel(xg.cpu().numpy(), xr)
    say(f"  reconstruction vs FP64-map oracle {e:.2e}")
    assert e < TOL                       # the primal never sees the rounded maps
    u = ut.cpu().numpy()
    for k in range(2):
        e = _rel(u[k], f.jvp(w[k], cr))
        say(f"  jvp probe {k} vs FP64-map oracle {e:.2e}")
        assert e < TOL_BF16
    ref = ocs.noise_map_jvp(f, cr, 21, 0, nprobe_map)["sum"].ravel()
    e, es = _rel(g, ref), _std_nrmse(g, ref)
    say(f"  |J w|^2 map ({nprobe_map} probes) vs FP64-map oracle: var {e:.2e}, std map {es:.2e}")
    assert e < TOL_BF16 and es < TOL_BF16


@pytest.mark.parametrize("storage", [1, 2])
def test_bf16_cs_jvp(lib, storage):
    say(f"case: CS L1-db4 64x64, 4 coils, Poisson-disc R=2, lam 1e-3, FISTA 30, 3 levels; recon, "
        f"2 JVPs and a 6-probe map, storage {storage}")
    maps, psi, mask, op, bw, braw = _cs_case(64, 64, 4, 3)
    h = lib.pico_init(64, 64, _dev(maps.astype(np.complex64)), psi, _dev(mask), sampling=lib.PICO_CART_2D,
                      recon=lib.PICO_CS_FISTA_L1WAV, kdata=_dev(braw.astype(np.complex64)), fista_iters=30,
                      cs_lambda=1e-3, wavelet_levels=3, probe_tile=2, storage=storage)
    try:
        _cs_check(lib, h, ocs.FistaL1Wavelet(op, 1e-3, 30, levels=3), op, bw, (64, 64))
    finally:
        lib.pico_destroy(h)


@pytest.mark.parametrize("storage", [1, 2])
def test_bf16_tv_cs_jvp(lib, storage):
    say(f"case: TV-CS 64x96, 4 coils, Poisson-disc R=2 (8x8 calib), lam_TV 1e-2, FISTA 30 x 10 dual "
        f"steps; recon, 2 JVPs and a 6-probe map, storage {storage}")
    maps, psi, mask, op, bw, braw = _cs_case(64, 96, 4, 5)
    h = lib.pico_init(64, 96, _dev(maps.astype(np.complex64)), psi, _dev(mask), sampling=lib.PICO_CART_2D,
                      recon=lib.PICO_CS_FISTA_TV, kdata=_dev(braw.astype(np.complex64)), fista_iters=30,
                      cs_lambda=1e-2, tv_inner_iters=10, probe_tile=2, storage=storage)
    try:
        _cs_check(lib, h, ocs.FistaTV(op, 1e-2, 30, 10), op, bw, (64, 96))
    finally:
        lib.pico_destroy(h)


@pytest.mark.parametrize("recon,nc,K", [("l1", 8, 128), ("tv", 15, 64)])
def test_bf16_cs_full_size_map_vs_fp32_storage(lib, recon, nc, K):
    tv = recon == "tv"
    say(f"case: {'TV' if tv else 'L1-db4'} CS 320x320, {nc} coils, Poisson-disc R=2 (24x24 calib), FISTA 100, "
        f"K={K} in one launch; noise map of bfloat16 maps + planes vs FP32 storage")
    maps, psi, mask, op, bw, braw = _cs_case(320, 320, nc, 11, calib=24)
    maps_t, mask_t, kd_t = _dev(maps.astype(np.complex64)), _dev(mask), _dev(braw.astype(np.complex64))
    kw = dict(sampling=lib.PICO_CART_2D, recon=lib.PICO_CS_FISTA_TV if tv else lib.PICO_CS_FISTA_L1WAV,
              kdata=kd_t, fista_iters=100, cs_lambda=1e-2 if tv else 1e-3, wavelet_levels=4,
              tv_inner_iters=10, probe_tile=K)
    maps_out = {}
    for storage in (0, 2):
        h = lib.pico_init(320, 320, maps_t, psi, mask_t, storage=storage, **kw)
        maps_out[storage] = _gpu_map(lib, h, 320 * 320, 31, 0, K)
        lib.pico_destroy(h)
    e, es = _rel(maps_out[2], maps_out[0]), _std_nrmse(maps_out[2], maps_out[0])
    say(f"  bfloat16 vs FP32 storage, {K} probes: variance map {e:.2e}, std map {es:.2e}")
    assert es < TOL_BF16 and e < TOL_BF16


def test_bf16_stream_spiral_full_size(lib):
    say("case: spiral 256x256, 16 coils, 48x4096 R=2 (98304 samples), lambda 0.1, CG 30, K=256 in one "
        "launch, bfloat16 maps and planes; apply_cov on probes 0 and 255 checked")
    prob = workloads.config(3, seed=0)
    traj = prob.traj.astype(np.float32)
    h = lib.pico_init(256, 256, _dev(prob.maps.astype(np.complex64)), prob.psi, None,
                      sampling=lib.PICO_NONCART, lam=0.1, cg_iters=30, probe_tile=256, traj=_dev(traj),
                      nsamples=traj.shape[0], storage=lib.PICO_BF16_STREAM)
    rng = np.random.default_rng(5)
    v = np.zeros((256, 256, 256), np.complex64)
    for k in (0, 255):
        v[k] = np.exp(2j * np.pi * rng.random((256, 256)))
    vt = _dev(v)
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 256)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cov = opico.Covariance(onufft.NonCartOp(prob.maps, prob.psi, traj.astype(np.float64)), 0.1, 30)
    u = ut[torch.tensor([0, 255], device="cuda:0")].cpu().numpy()
    for j, k in enumerate((0, 255)):
        e = _rel(u[j], cov.apply(v[k].astype(np.complex128)))
        say(f"  probe {k}: vs FP64 oracle {e:.2e}")
        assert e < TOL_BF16
