"""GPU parity of the 2-D grid path (Cartesian 2-D masks and the spiral
Toeplitz operator) against the FP64 oracle on the same seeded probes.

The GPU receives the trajectory in float32; the oracle is fed the same
float32-rounded trajectory so that both sides define the same operator.
Bar: relative 2-norm error <= 1e-4 (float32 storage).
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import nufft as onufft
from oracle import pico as opico
from oracle import storage as ostore

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


def _gpu_map(lib, h, n, seed, first, nprobes, stats=None):
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    acc = lib.make_accum(*acc_t)
    lib.pico_noise_map(h, seed, first, nprobes, 0, acc, stats)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in acc_t]


def _spiral_problem(n=64, nc=4, R=2, inter=16, samples=512, seed=3, lam=0.1, cg=20):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n, n, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    traj = workloads.spiral_traj(n, R, inter, samples).astype(np.float32)
    return maps, psi, traj, lam, cg


def _init_noncart(lib, maps, psi, traj, lam, cg, tile):
    n = maps.shape[1]
    return lib.pico_init(n, n, _dev(maps.astype(np.complex64)), psi, None,
                         sampling=lib.PICO_NONCART, lam=lam, cg_iters=cg, probe_tile=tile,
                         traj=_dev(traj), nsamples=traj.shape[0])


def test_cart2d_poisson_disc_parity(lib):
    say("case: Cartesian 2-D Poisson-disc mask 96x64, 5 coils, 6 probes in tiles of 4, CG 20")
    rng = np.random.default_rng(11)
    maps = workloads.coil_maps(96, 64, 5, rng)
    psi = workloads.noise_cov(5, rng)
    mask = workloads.poisson_disc_mask(96, 64, 2.0, 12, seed=1)
    h = lib.pico_init(96, 64, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                      sampling=lib.PICO_CART_2D, cg_iters=20, probe_tile=4)
    st = lib.pico_stats_t()
    s, si, ss = _gpu_map(lib, h, 96 * 64, 5, 2, 6, st)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(maps, psi, mask), 0.0, 20)
    ref = opico.noise_map(cov, 5, 2, 6)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err {err:.2e}; CG relres max {st.max_relres:.2e}")
    assert err < TOL
    assert _rel(ss, ref["sumsq"].ravel()) < TOL


def test_cart2d_tikhonov_apply_cov(lib):
    say("case: Cartesian 2-D uniform 2x2 mask 64x64, lambda 0.05, apply_cov on 2 probes")
    rng = np.random.default_rng(12)
    maps = workloads.coil_maps(64, 64, 6, rng)
    psi = workloads.noise_cov(6, rng)
    mask = workloads.cart_mask_2d_uniform(64, 64, 2, 2)
    h = lib.pico_init(64, 64, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                      sampling=lib.PICO_CART_2D, lam=0.05, cg_iters=25, probe_tile=2)
    v = np.stack([opico.probe_image(3, i, (64, 64)) for i in range(2)])
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 2)
    torch.cuda.synchronize()
    lam_abs = lib.pico_lambda_abs(h)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(maps, psi, mask), 0.05, 25)
    assert abs(lam_abs - cov.lam) < 1e-5 * cov.lam
    u = ut.cpu().numpy()
    for k in range(2):
        err = _rel(u[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {err:.2e}")
        assert err < TOL


def test_spiral_toeplitz_noise_map_parity(lib):
    say("case: spiral Toeplitz 64x64, 4 coils, 16x512 R=2, lambda 0.1, 6 probes in tiles of 4")
    maps, psi, traj, lam, cg = _spiral_problem()
    h = _init_noncart(lib, maps, psi, traj, lam, cg, 4)
    st = lib.pico_stats_t()
    s, _, _ = _gpu_map(lib, h, 64 * 64, 9, 0, 6, st)
    lam_abs = lib.pico_lambda_abs(h)
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64))
    cov = opico.Covariance(op, lam, cg)
    say(f"  lambda_abs gpu {lam_abs:.8e} oracle {cov.lam:.8e}")
    assert abs(lam_abs - cov.lam) < 1e-5 * cov.lam
    ref = opico.noise_map(cov, 9, 0, 6)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err {err:.2e}; CG relres max {st.max_relres:.2e}")
    assert err < TOL


def test_spiral_toeplitz_nonsquare_grid(lib):
    # lambda > 0: a spiral samples a disc of k-space, so at lambda = 0 the
    # normal operator is singular (its corners are in the null space)
    say("case: spiral Toeplitz 48x80 (grid 96x160), 3 coils, lambda 0.05, apply_cov 3 probes")
    rng = np.random.default_rng(5)
    maps = workloads.coil_maps(48, 80, 3, rng)
    psi = workloads.noise_cov(3, rng)
    traj = workloads.spiral_traj(80, 1, 12, 600).astype(np.float32)
    h = lib.pico_init(48, 80, _dev(maps.astype(np.complex64)), psi, None,
                      sampling=lib.PICO_NONCART, lam=0.05, cg_iters=40, probe_tile=3,
                      traj=_dev(traj), nsamples=traj.shape[0])
    v = np.stack([opico.probe_image(1, i, (48, 80)) for i in range(3)])
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 3)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64))
    cov = opico.Covariance(op, 0.05, 40)
    u = ut.cpu().numpy()
    for k in range(3):
        err = _rel(u[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {err:.2e}")
        assert err < TOL


@pytest.mark.parametrize("R", [2, 3, 4])
def test_spiral_full_size_sampled_probes(lib, R):
    checked = (0, 137, 255) if R == 2 else (255,)
    say(f"case: spiral 256x256, 16 coils, 48x4096 R={R} ({98304 * 2 // R} samples), lambda 0.1, CG 30, "
        f"K=256 right-hand sides in one launch; probes {checked} checked, every probe by property")
    prob = workloads.config(3, seed=0, R=R)
    traj = prob.traj.astype(np.float32)
    h = _init_noncart(lib, prob.maps, prob.psi, traj, prob.lam, prob.cg_iters, 256)
    v = np.stack([opico.probe_image(42, i, (256, 256)) for i in range(256)]).astype(np.complex64)
    vt = _dev(v)
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 256)
    torch.cuda.synchronize()
    lam_abs = lib.pico_lambda_abs(h)
    lib.pico_destroy(h)
    u = ut.cpu().numpy()
    op = onufft.NonCartOp(prob.maps, prob.psi, traj.astype(np.float64))
    cov = opico.Covariance(op, prob.lam, prob.cg_iters)
    say(f"  lambda_abs gpu {lam_abs:.8e} oracle {cov.lam:.8e}")
    for k in checked:
        ref = cov.apply(v[k].astype(np.complex128))
        err = _rel(u[k], ref)
        vox = float(np.max(np.abs(u[k] - ref)) / np.max(np.abs(ref)))
        say(f"  probe {k}: rel err {err:.2e}, max voxel error / max |ref| {vox:.2e}")
        assert err < TOL and vox < 10 * TOL
    # every right-hand side of the launch: Sigma = (M + l)^-1 M (M + l)^-1 is
    # Hermitian with eigenvalues t / (t + l)^2 in [0, 1 / (4 l)], so
    # 0 < Re <v, Sigma v> <= |v|^2 / (4 l) and Im <v, Sigma v> = 0 (to rounding)
    q = np.einsum("kyx,kyx->k", np.conj(v.astype(np.complex128)), u.astype(np.complex128))
    vv = np.sum(np.abs(v.astype(np.complex128)) ** 2, axis=(1, 2))
    assert np.all(q.real > 0)
    assert np.all(q.real <= vv / (4 * lam_abs) * (1 + 1e-4))
    assert np.max(np.abs(q.imag) / q.real) < 1e-4
    say(f"  all 256 probes: Re<v, u> / |v|^2 in [{(q.real / vv).min():.3e}, {(q.real / vv).max():.3e}] "
        f"(bound {1 / (4 * lam_abs):.3e}), max |Im| / Re {np.max(np.abs(q.imag) / q.real):.1e}")


# Line lengths with two-step plans whose lane groups do not divide a
# wavefront evenly (18 and 24 lanes) or fill it (32 lanes), and the 64-lane
# Stockham plan of 768 points.  Row counts are chosen so that the last
# workgroup of the row passes holds a partial set of row groups.
@pytest.mark.parametrize("kind,ny,nx,storage", [
    ("spiral", 128, 144, 0),   # rows 288 (three 18-lane groups; 2 x 128 rows: ragged), columns 256
    ("spiral", 144, 96, 0),    # columns 288
    ("spiral", 192, 160, 0),   # rows 320 x columns 384
    ("spiral", 96, 192, 2),    # rows 384 (two 24-lane groups), bfloat16 maps and planes
    ("spiral", 288, 320, 0),   # rows 640 x columns 576
    ("spiral", 320, 288, 2),   # rows 576 x columns 640, bfloat16 maps and planes
    ("cart2d", 160, 288, 0),   # Cartesian rows 288 (2 x 160 rows: ragged over groups of 3)
    ("cart2d", 384, 384, 0),   # Cartesian rows and columns 384
    ("spiral", 96, 64, 0),     # rows 128 x columns 192
    ("cart2d", 192, 160, 0),   # Cartesian rows 160 x columns 192
    ("cart2d", 96, 96, 2),     # Cartesian rows and columns 96 (five 12-lane groups), bfloat16
])
def test_grid_line_lengths(lib, kind, ny, nx, storage):
    K = 2
    say(f"case: {kind} {ny}x{nx}, 2 coils, storage {storage}, apply_cov on {K} probes in one tile, CG 15")
    rng = np.random.default_rng(ny * 1000 + nx)
    maps = workloads.coil_maps(ny, nx, 2, rng)
    psi = workloads.noise_cov(2, rng)
    if kind == "spiral":
        traj = workloads.spiral_traj(max(ny, nx), 1, 12, 1024).astype(np.float32)
        h = lib.pico_init(ny, nx, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART,
                          lam=0.1, cg_iters=15, probe_tile=K, traj=_dev(traj), nsamples=traj.shape[0],
                          storage=storage)
        lam = 0.1
        op_maps = ostore.bf16_whitened_maps(maps, psi) if storage else maps
        op = onufft.NonCartOp(op_maps, None if storage else psi, traj.astype(np.float64))
    else:
        mask = workloads.poisson_disc_mask(ny, nx, 2.0, 16, seed=ny + nx)
        h = lib.pico_init(ny, nx, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                          sampling=lib.PICO_CART_2D, lam=0.05, cg_iters=15, probe_tile=K, storage=storage)
        lam = 0.05
        op = opico.cartesian(maps, psi, mask)
    v = np.stack([opico.probe_image(7, i, (ny, nx)) for i in range(K)])
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, K)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cov = opico.Covariance(op, lam, 15)
    # storage 2 rounds every plane to bfloat16 as well: the rounded-map oracle
    # bounds the map rounding only, so the bar is the bfloat16 one
    tol = TOL if storage == 0 else 1e-2
    u = ut.cpu().numpy()
    for k in range(K):
        err = _rel(u[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {err:.2e}")
        assert err < tol
