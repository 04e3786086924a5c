"""GPU parity of the Kaiser-Bessel gridding data path of non-Cartesian
operators (A and A^H through pico_apply_nufft) and of PMR on spiral sampling,
against the FP64 oracle's gridding NUFFT with the same parameters."""
import sys

import numpy as np
import pytest

import workloads
from oracle import nufft as onufft
from oracle import pico as opico

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


def _setup(n, nc, R, inter, samples, seed):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n, n, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    traj = workloads.spiral_traj(n, R, inter, samples).astype(np.float32)
    return rng, maps, psi, traj


def _init(lib, maps, psi, traj, sigma, W, tile, lam=0.1, cg=20):
    n = maps.shape[1]
    return lib.pico_init(n, n, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART,
                         lam=lam, cg_iters=cg, probe_tile=tile, traj=_dev(traj), nsamples=traj.shape[0],
                         oversamp=sigma, kb_width=W)


@pytest.mark.parametrize("n,nc,sigma,W,samples", [(64, 4, 2.0, 6, 512), (128, 3, 1.25, 4, 1024)])
def test_gridding_forward_adjoint_parity(lib, n, nc, sigma, W, samples):
    say(f"case: gridding {n}x{n}, {nc} coils, sigma {sigma}, W {W}, 16 interleaves x {samples}, k=3")
    rng, maps, psi, traj = _setup(n, nc, 2, 16, samples, seed=5)
    M = traj.shape[0]
    h = _init(lib, maps, psi, traj, sigma, W, 4)
    x = (rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))).astype(np.complex64)
    y = (rng.standard_normal((3, nc, M)) + 1j * rng.standard_normal((3, nc, M))).astype(np.complex64)
    fo = torch.empty((3, nc, M), dtype=torch.complex64, device="cuda:0")
    ad = torch.empty((3, n, n), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_nufft(h, 0, _dev(x), fo, 3)
    lib.pico_apply_nufft(h, 1, _dev(y), ad, 3)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64), kb=(sigma, W))
    for k in range(3):
        ef = _rel(fo.cpu().numpy()[k], op.forward(x[k].astype(np.complex128)))
        ea = _rel(ad.cpu().numpy()[k], op.adjoint(y[k].astype(np.complex128)))
        say(f"  image {k}: forward rel err {ef:.2e}, adjoint rel err {ea:.2e}")
        assert ef < TOL and ea < TOL


def test_spiral_pmr_parity(lib):
    say("case: PMR on spiral 64x64, 4 coils, 16x512 R=2, gridding sigma 2 W 6, lambda 0.1, "
        "CG 20, 10 replicas in tiles of 4")
    rng, maps, psi, traj = _setup(64, 4, 2, 16, 512, seed=8)
    h = _init(lib, maps, psi, traj, 2.0, 6, 4)
    n = 64 * 64
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lib.pico_pmr_baseline(h, 13, 3, 10, lib.make_accum(*acc_t))
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64), kb=(2.0, 6))
    ref = opico.pmr(opico.Covariance(op, 0.1, 20), 13, 3, 10)
    for key, t in zip(("sum", "sum_im", "sumsq"), acc_t):
        e = _rel(t.cpu().numpy(), ref[key].ravel())
        say(f"  {key}: rel err {e:.2e}")
        assert e < TOL


@pytest.mark.parametrize("sigma,W", [(2.0, 6), (1.25, 4)])
def test_gridding_full_size(lib, sigma, W):
    say(f"case: gridding at the spiral workload's size: 256x256, 16 coils, 48x4096 R=2 "
        f"(98304 samples), sigma {sigma}, W {W}, k=2")
    rng, maps, psi, traj = _setup(256, 16, 2, 48, 4096, seed=0)
    M = traj.shape[0]
    h = _init(lib, maps, psi, traj, sigma, W, 2, cg=30)
    x = (rng.standard_normal((2, 256, 256)) + 1j * rng.standard_normal((2, 256, 256))).astype(np.complex64)
    y = (rng.standard_normal((2, 16, M)) + 1j * rng.standard_normal((2, 16, M))).astype(np.complex64)
    fo = torch.empty((2, 16, M), dtype=torch.complex64, device="cuda:0")
    ad = torch.empty((2, 256, 256), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_nufft(h, 0, _dev(x), fo, 2)
    lib.pico_apply_nufft(h, 1, _dev(y), ad, 2)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64), kb=(sigma, W))
    for k in range(2):
        ef = _rel(fo.cpu().numpy()[k], op.forward(x[k].astype(np.complex128)))
        ea = _rel(ad.cpu().numpy()[k], op.adjoint(y[k].astype(np.complex128)))
        say(f"  image {k}: forward rel err {ef:.2e}, adjoint rel err {ea:.2e}")
        assert ef < TOL and ea < TOL


@pytest.mark.parametrize("n,nc,sigma,W,samples", [(64, 4, 2.0, 6, 512), (128, 3, 1.25, 4, 1024),
                                                  (64, 3, 2.0, 2, 512), (64, 3, 2.0, 8, 512)])
def test_gridding_normal_operator_parity(lib, n, nc, sigma, W, samples):
    say(f"case: CG on the gridding normal operator (binned tile interp/spread), {n}x{n}, {nc} coils, "
        f"sigma {sigma}, W {W}, 16 x {samples} R=2, lambda 0.1, CG 20; apply_cov on 3 probes and a "
        "7-probe map in tiles of 3")
    rng, maps, psi, traj = _setup(n, nc, 2, 16, samples, seed=n + W)
    h = lib.pico_init(n, n, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART, lam=0.1,
                      cg_iters=20, probe_tile=3, traj=_dev(traj), nsamples=traj.shape[0], oversamp=sigma,
                      kb_width=W, noncart_normal=1)
    v = np.stack([opico.probe_image(3, i, (n, n)) for i in range(3)]).astype(np.complex64)
    ut = torch.empty((3, n, n), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_cov(h, _dev(v), ut, 3)
    acc_t = [torch.zeros(n * n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lib.pico_noise_map(h, 9, 2, 7, 0, lib.make_accum(*acc_t))
    lam_abs = lib.pico_lambda_abs(h)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64), kb=(sigma, W), normal_mode="gridding")
    cov = opico.Covariance(op, 0.1, 20)
    say(f"  lambda_abs gpu {lam_abs:.8e} oracle {cov.lam:.8e}")
    assert abs(lam_abs - cov.lam) <= 1e-5 * cov.lam
    u = ut.cpu().numpy()
    for k in range(3):
        e = _rel(u[k], cov.apply(v[k].astype(np.complex128)))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL
    ref = opico.noise_map(cov, 9, 2, 7)
    for key, t in zip(("sum", "sum_im", "sumsq"), acc_t):
        e = _rel(t.cpu().numpy(), ref[key].ravel())
        say(f"  map {key}: rel err {e:.2e}")
        assert e < TOL


# Non-square images: the image rows (ny) and columns (nx) sit on grids of
# different lengths, so a swap of the two in the row and column passes of the
# gridding normal operator shows here
@pytest.mark.parametrize("ny,nx,W", [(64, 96, 6), (96, 64, 4)])
def test_gridding_normal_operator_nonsquare(lib, ny, nx, W):
    say(f"case: CG on the gridding normal operator, {ny}x{nx} (grid {2 * ny}x{2 * nx}), 3 coils, sigma 2, "
        f"W {W}, 16 x 512 R=2, lambda 0.1, CG 20; apply_cov on 2 probes and a 4-probe map in tiles of 2")
    rng = np.random.default_rng(ny + nx + W)
    maps = workloads.coil_maps(ny, nx, 3, rng)
    psi = workloads.noise_cov(3, rng)
    traj = workloads.spiral_traj(max(ny, nx), 2, 16, 512).astype(np.float32)
    h = lib.pico_init(ny, nx, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART, lam=0.1,
                      cg_iters=20, probe_tile=2, traj=_dev(traj), nsamples=traj.shape[0], oversamp=2.0,
                      kb_width=W, noncart_normal=1)
    v = np.stack([opico.probe_image(5, i, (ny, nx)) for i in range(2)]).astype(np.complex64)
    ut = torch.empty((2, ny, nx), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_cov(h, _dev(v), ut, 2)
    acc_t = [torch.zeros(ny * nx, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lib.pico_noise_map(h, 11, 0, 4, 0, lib.make_accum(*acc_t))
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64), kb=(2.0, W), normal_mode="gridding")
    cov = opico.Covariance(op, 0.1, 20)
    u = ut.cpu().numpy()
    for k in range(2):
        e = _rel(u[k], cov.apply(v[k].astype(np.complex128)))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL
    ref = opico.noise_map(cov, 11, 0, 4)
    e = _rel(acc_t[0].cpu().numpy(), ref["sum"].ravel())
    say(f"  map sum: rel err {e:.2e}")
    assert e < TOL


def test_gridding_normal_full_size_vs_toeplitz(lib):
    say("case: spiral 256x256, 16 coils, 48x4096 R=2, lambda 0.1, CG 30, K=256 in one launch: "
        "Sigma v with the gridding normal operator (sigma 2, W 6) against the exact Toeplitz one")
    rng, maps, psi, traj = _setup(256, 16, 2, 48, 4096, seed=0)
    v = np.stack([opico.probe_image(42, i, (256, 256)) for i in range(256)]).astype(np.complex64)
    vt = _dev(v)
    out = {}
    for mode in (0, 1):
        h = lib.pico_init(256, 256, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART,
                          lam=0.1, cg_iters=30, probe_tile=256, traj=_dev(traj), nsamples=traj.shape[0],
                          oversamp=2.0, kb_width=6, noncart_normal=mode)
        ut = torch.empty_like(vt)
        lib.pico_apply_cov(h, vt, ut, 256)
        torch.cuda.synchronize()
        out[mode] = ut.cpu().numpy()
        lib.pico_destroy(h)
    e = np.array([_rel(out[1][k], out[0][k]) for k in range(256)])
    say(f"  ||Sigma_grid v - Sigma_T v|| / ||Sigma_T v|| over 256 probes: max {e.max():.2e}, mean {e.mean():.2e}")
    assert np.all(np.isfinite(out[1])) and e.max() < 1e-3
