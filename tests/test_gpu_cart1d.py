"""GPU parity of the separable Cartesian path (libpico through its C ABI)
against the FP64 oracle on the same seeded probes.

Bar (single precision storage): relative 2-norm error <= 1e-4 of the
variance map (and of u = Sigma v), per the path's stated tolerance.
"""
import sys

import numpy as np
import pytest

import workloads
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


def _init(lib, prob, tile, lam=None, cg_iters=None, cg_tol=0.0, form=0):
    maps = _dev(prob.maps.astype(np.complex64))
    mask = _dev(prob.mask)
    return lib.pico_init(prob.ny, prob.nx, maps, prob.psi, mask,
                         lam=prob.lam if lam is None else lam,
                         cg_iters=prob.cg_iters if cg_iters is None else cg_iters,
                         cg_tol=cg_tol, probe_tile=tile, normal_form=form)


def _gpu_map(lib, h, n, seed, first, nprobes, dist=0, stats=None, acc_t=None):
    if acc_t is None:
        acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    acc = lib.make_accum(*acc_t)
    lib.pico_noise_map(h, seed, first, nprobes, dist, acc, stats)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in acc_t], acc


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_config1_noise_map_parity(lib):
    say("case: config-1 64x64 4 coils R=2, 16 probes, CG 20, tile 16")
    prob = workloads.config(1, seed=0)
    h = _init(lib, prob, 16)
    (s, si, ss), _ = _gpu_map(lib, h, prob.ny * prob.nx, 77, 0, 16)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, prob.cg_iters)
    ref = opico.noise_map(cov, 77, 0, 16)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err sum {err:.2e}, max voxel rel {np.max(np.abs(s - ref['sum'].ravel()) / np.abs(ref['sum'].ravel())):.2e}")
    assert err < TOL
    assert _rel(ss, ref["sumsq"].ravel()) < TOL
    assert np.abs(si - ref["sum_im"].ravel()).max() < TOL * np.abs(ref["sum"]).max()


@pytest.mark.parametrize("dist", ["qpsk", "rademacher", "gaussian"])
def test_probe_families_parity(lib, dist):
    say(f"case: config-1 probe family {dist}, 4 probes")
    prob = workloads.config(1, seed=2)
    h = _init(lib, prob, 4)
    (s, _, _), _ = _gpu_map(lib, h, prob.ny * prob.nx, 5, 3, 4, dist=lib.PROBES[dist])
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, prob.cg_iters)
    ref = opico.noise_map(cov, 5, 3, 4, dist=dist)
    assert _rel(s, ref["sum"].ravel()) < TOL


def test_ragged_tiles_and_odd_width(lib):
    say("case: 96x40 5 coils R=2 + 8 ACS, 10 probes in tiles of 4 (4+4+2), CG 25")
    prob = workloads.config(2, seed=3, ny=96, nx=40, nc=5, acs=8, cg_iters=25)
    h = _init(lib, prob, 4)
    st = lib.pico_stats_t()
    (s, _, ss), acc = _gpu_map(lib, h, prob.ny * prob.nx, 11, 7, 10, stats=st)
    lib.pico_destroy(h)
    assert acc.count == 10 and st.probes == 10 and st.frozen == 0
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, prob.cg_iters)
    ref = opico.noise_map(cov, 11, 7, 10)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err {err:.2e}, CG max relres {st.max_relres:.2e}")
    assert err < TOL


def test_apply_cov_parity_and_tikhonov(lib):
    say("case: apply_cov on 3 explicit probes, lambda 0 and 0.1, 64x64")
    prob = workloads.config(1, seed=4)
    rng = np.random.default_rng(8)
    v = (rng.standard_normal((3, 64, 64)) + 1j * rng.standard_normal((3, 64, 64)))
    for lam in (0.0, 0.1):
        h = _init(lib, prob, 4, lam=lam, cg_iters=30)
        vt = _dev(v.astype(np.complex64))
        ut = torch.empty_like(vt)
        lib.pico_apply_cov(h, vt, ut, 3)
        torch.cuda.synchronize()
        lam_abs = lib.pico_lambda_abs(h)
        lib.pico_destroy(h)
        cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), lam, 30)
        if lam > 0:
            say(f"  lambda_abs gpu {lam_abs:.8e} oracle {cov.lam:.8e}")
            assert abs(lam_abs - cov.lam) < 1e-5 * cov.lam
        u = ut.cpu().numpy()
        for k in range(3):
            ref = cov.apply(v[k])
            err = _rel(u[k], ref)
            say(f"  lambda {lam} probe {k}: rel err {err:.2e}")
            assert err < TOL


@pytest.mark.parametrize("form", [0, 3])
def test_cg_tolerance_mode_parity(lib, form):
    say(f"case: CG to ||r||/||r0|| <= 1e-5 (at most 200 iterations), 96x40 5 coils R=2 + 8 ACS, "
        f"12 probes in tiles of 8, normal form {form}")
    prob = workloads.config(2, seed=8, ny=96, nx=40, nc=5, acs=8, cg_iters=200)
    h = _init(lib, prob, 8, cg_tol=1e-5, form=form)
    st = lib.pico_stats_t()
    (s, _, _), _ = _gpu_map(lib, h, prob.ny * prob.nx, 13, 0, 12, stats=st)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 200, tol=1e-5)
    ref = opico.noise_map(cov, 13, 0, 12)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err {err:.2e}, CG relres max {st.max_relres:.2e}, frozen {st.frozen}")
    # every solve stopped by the tolerance; a stop one iteration apart from the
    # oracle's moves x by ~1e-5 relative, far inside the bar
    assert st.max_relres <= 1e-5 and st.frozen == 0
    assert err < TOL


def test_tikhonov_noise_map_parity(lib):
    say("case: Tikhonov lambda 0.1 noise map, 128x48 6 coils, 6 probes")
    prob = workloads.config(2, seed=5, ny=128, nx=48, nc=6, acs=8, cg_iters=20, lam=0.1)
    h = _init(lib, prob, 8)
    (s, _, _), _ = _gpu_map(lib, h, prob.ny * prob.nx, 3, 0, 6)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.1, prob.cg_iters)
    ref = opico.noise_map(cov, 3, 0, 6)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("form", [0, 3])
def test_resume_split_is_bitwise(lib, form):
    say(f"case: probes [0,8)+[8,16) vs [0,16), tile 8, normal form {form}")
    prob = workloads.config(1, seed=6)
    n = prob.ny * prob.nx
    h = _init(lib, prob, 8, form=form)
    (a, _, _), _ = _gpu_map(lib, h, n, 9, 0, 16)
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    _gpu_map(lib, h, n, 9, 0, 8, acc_t=acc_t)
    (b, _, _), _ = _gpu_map(lib, h, n, 9, 8, 8, acc_t=acc_t)
    lib.pico_destroy(h)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("form", [0, 3])
def test_pmr_parity(lib, form):
    say(f"case: PMR 24 replicas, 64x64 4 coils, tile 8, normal form {form}")
    prob = workloads.config(1, seed=7)
    n = prob.ny * prob.nx
    h = _init(lib, prob, 8, form=form)
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    acc = lib.make_accum(*acc_t)
    lib.pico_pmr_baseline(h, 21, 0, 24, acc)
    var = torch.empty(n, dtype=torch.float64, device="cuda:0")
    lib.pico_pmr_finalize(h, acc, var)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, prob.cg_iters)
    ref = opico.pmr(cov, 21, 0, 24)
    for key, t in zip(("sum", "sum_im", "sumsq"), acc_t):
        err = _rel(t.cpu().numpy(), ref[key].ravel())
        say(f"  PMR {key}: rel err {err:.2e}")
        assert err < TOL
    assert _rel(var.cpu().numpy(), opico.pmr_finalize(ref).ravel()) < TOL


def test_full_size_config2_all_columns(lib):
    say("case: config-2 320x320 15 coils R=2+24 ACS, K=256 probes as one tile, CG 30, "
        "dense (matrix-core) and FFT normal forms; every column against the converged oracle")
    prob = workloads.config(2, seed=0)
    n = prob.ny * prob.nx
    op = opico.cartesian(prob.maps, prob.psi, prob.mask)
    cols = list(range(prob.nx))
    ref = opico.noise_map_exact_columns(op, prob.mask, 2024, 0, 256, cols)
    for form, name in ((2, "dense"), (3, "dense split-FP16"), (1, "FFT")):
        h = _init(lib, prob, 256, form=form)
        st = lib.pico_stats_t()
        (s, _, _), acc = _gpu_map(lib, h, n, 2024, 0, 256, stats=st)
        lib.pico_destroy(h)
        say(f"  {name}: CG relres max {st.max_relres:.2e} mean {st.mean_relres:.2e}, frozen {st.frozen}")
        assert st.frozen == 0 and acc.count == 256
        got = s.reshape(prob.ny, prob.nx)[:, cols]
        err = _rel(got, ref)
        vox = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        say(f"  {name}: all {len(cols)} columns: rel err vs converged oracle {err:.2e}, "
            f"max voxel error / max |ref| {vox:.2e}")
        assert err < TOL and vox < 10 * TOL


@pytest.mark.parametrize("form", [2, 3])
@pytest.mark.parametrize("ny,nx,nc,tile,nprobes", [(64, 64, 4, 40, 40), (96, 40, 5, 4, 10),
                                                   (160, 24, 8, 32, 45), (288, 16, 3, 33, 33),
                                                   (512, 8, 2, 32, 32)])
def test_dense_form_parity(lib, ny, nx, nc, tile, nprobes, form):
    say(f"case: dense per-column normal operator (form {form}) {ny}x{nx} {nc} coils, {nprobes} probes "
        f"in tiles of {tile} (probe tiles of 32 on the matrix cores, ragged), CG 20")
    prob = workloads.config(2, seed=ny, ny=ny, nx=nx, nc=nc, acs=8, cg_iters=20)
    h = _init(lib, prob, tile, form=form)
    st = lib.pico_stats_t()
    (s, si, ss), _ = _gpu_map(lib, h, ny * nx, 31, 2, nprobes, stats=st)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 20)
    ref = opico.noise_map(cov, 31, 2, nprobes)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err sum {err:.2e}, sumsq {_rel(ss, ref['sumsq'].ravel()):.2e}, CG relres max {st.max_relres:.2e}")
    assert err < TOL and _rel(ss, ref["sumsq"].ravel()) < TOL


# Column transforms of every line length on the FFT path (normal form 0):
# two-step plans whose lane groups leave part of the wavefront idle (12 lanes
# at 96, 18 at 288, 24 at 384) or fill it, and the 64-lane Stockham plan of
# 512 points, with ragged probe tiles.
@pytest.mark.parametrize("ny,nx,nc,tile,nprobes", [(96, 40, 5, 4, 10), (128, 24, 6, 9, 9),
                                                   (160, 24, 8, 32, 45),
                                                   (192, 20, 4, 7, 7), (288, 16, 3, 33, 33),
                                                   (384, 12, 3, 17, 17), (512, 8, 2, 32, 32)])
def test_fft_form_column_lengths(lib, ny, nx, nc, tile, nprobes):
    say(f"case: FFT normal form {ny}x{nx} {nc} coils, {nprobes} probes in tiles of {tile}, CG 20")
    prob = workloads.config(2, seed=ny + 1, ny=ny, nx=nx, nc=nc, acs=8, cg_iters=20)
    h = _init(lib, prob, tile, form=0)
    st = lib.pico_stats_t()
    (s, si, ss), _ = _gpu_map(lib, h, ny * nx, 33, 1, nprobes, stats=st)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 20)
    ref = opico.noise_map(cov, 33, 1, nprobes)
    err = _rel(s, ref["sum"].ravel())
    say(f"  rel err sum {err:.2e}, sumsq {_rel(ss, ref['sumsq'].ravel()):.2e}, CG relres max {st.max_relres:.2e}")
    assert err < TOL and _rel(ss, ref["sumsq"].ravel()) < TOL


@pytest.mark.parametrize("form", [2, 3])
def test_dense_form_apply_cov_tikhonov(lib, form):
    say(f"case: dense normal form {form}, apply_cov on 3 probes, lambda 0.1, 64x64, power method on the "
        "matrix cores")
    prob = workloads.config(1, seed=4)
    rng = np.random.default_rng(8)
    v = (rng.standard_normal((3, 64, 64)) + 1j * rng.standard_normal((3, 64, 64)))
    h = _init(lib, prob, 4, lam=0.1, cg_iters=30, form=form)
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 3)
    torch.cuda.synchronize()
    lam_abs = lib.pico_lambda_abs(h)
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.1, 30)
    say(f"  lambda_abs gpu {lam_abs:.8e} oracle {cov.lam:.8e}")
    assert abs(lam_abs - cov.lam) < 1e-5 * cov.lam
    u = ut.cpu().numpy()
    for k in range(3):
        err = _rel(u[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {err:.2e}")
        assert err < TOL


def test_degenerate_single_coil_full_sampling(lib):
    say("case: 1 coil of unit magnitude, full sampling, psi = 2: Sigma = 2 I, 2 probes")
    yy, xx = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    maps = np.exp(2j * np.pi * (0.1 * yy + 0.03 * xx))[None]
    prob = workloads.Problem("deg", 64, 64, maps, np.array([[2.0]]), "cart1d",
                             mask=np.ones(64, np.uint8), cg_iters=5, probes=2)
    h = _init(lib, prob, 2)
    (s, si, ss), _ = _gpu_map(lib, h, 64 * 64, 1, 0, 2)
    lib.pico_destroy(h)
    # one random-phase probe is exact when Sigma is diagonal (kappa = 1)
    assert np.abs(s / 2 - 2.0).max() < 1e-5
    assert np.abs(si).max() < 1e-5


def test_exact_diag_and_monitor(lib):
    say("case: exact diagonal by row probing + NRMSE monitor, 160x24 8 coils R=2 + 16 ACS")
    from oracle import sense
    prob = workloads.config(2, seed=1, ny=160, nx=24, nc=8, acs=16, cg_iters=40)
    n = prob.ny * prob.nx
    h = _init(lib, prob, 64)
    ref = torch.empty(n, dtype=torch.float64, device="cuda:0")
    lib.pico_exact_diag(h, ref)
    (s, _, _), acc = _gpu_map(lib, h, n, 4, 0, 24)
    acc_t = [torch.from_numpy(s).to("cuda:0")]
    acc2 = lib.make_accum(acc_t[0], count=24)
    e_gpu = lib.pico_monitor_nrmse(h, acc2, ref)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = opico.cartesian(prob.maps, prob.psi, prob.mask)
    ex = sense.exact_diag_1d(op, prob.mask).ravel()
    err = _rel(ref.cpu().numpy(), ex)
    e_ref = opico.nrmse_std(s / 24, ex)
    say(f"  exact diag rel err {err:.2e}; monitor NRMSE gpu {e_gpu:.6f} oracle {e_ref:.6f}")
    assert err < TOL
    assert abs(e_gpu - e_ref) < 1e-6


def test_stderr_proxy_and_adaptive_stopping(lib):
    say("case: reference-free error proxy and adaptive stopping, 160x24 8 coils R=2 + 16 ACS, tiles of 16")
    prob = workloads.config(2, seed=1, ny=160, nx=24, nc=8, acs=16, cg_iters=40)
    n = prob.ny * prob.nx
    h = _init(lib, prob, 16)
    (s, si, ss), acc = _gpu_map(lib, h, n, 9, 0, 48)
    px = lib.pico_monitor_stderr(h, acc)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 40)
    ref = opico.noise_map(cov, 9, 0, 48)
    p_ref = opico.stderr_proxy(ref)
    say(f"  proxy gpu {px:.6f} oracle {p_ref:.6f}")
    assert abs(px - p_ref) < 1e-4 * p_ref
    # adaptive run to a 5 % proxy; check the std-map NRMSE against the exact map
    ex = torch.empty(n, dtype=torch.float64, device="cuda:0")
    lib.pico_exact_diag(h, ex)
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    acc2 = lib.make_accum(*acc_t)
    used, pfin = lib.pico_noise_map_adaptive(h, 17, 0, 4096, 0.05, 0, acc2)
    err = lib.pico_monitor_nrmse(h, acc2, ex)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    say(f"  adaptive: stopped at N={used} with proxy {pfin:.4f}; NRMSE vs exact {err:.4f}")
    assert used % 16 == 0 and used < 4096 and pfin <= 0.05
    assert err < 0.075
