"""GPU parity of the TV-regularised compressed-sensing path (the model of the
paper's CS experiment, Sec. 3.2.3: FISTA with an isotropic TV prox solved by
dual fast gradient projection), its Jacobian probes and its PMR replicas,
against the FP64 oracle (oracle.cs.FistaTV).

Image sizes are the 2-D FFT lengths the Cartesian path is built for, square
and not.
Inputs: k-space b = A x + noise from the oracle's whitened forward operator,
un-whitened (b_raw = L b_w) because the library whitens raw data itself.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import cs as ocs
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


def _setup(ny, nx, nc, R, calib, seed, snr_db=45.0):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(ny, nx, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    x = workloads.phantom(max(ny, nx), rng)[:ny, :nx]
    mask = workloads.poisson_disc_mask(ny, nx, R, calib, seed=seed)
    op = opico.cartesian(maps, psi, mask)
    bw = op.forward(x)
    sig = np.sqrt(np.mean(np.abs(bw[:, mask > 0]) ** 2)) * 10 ** (-snr_db / 20)
    noise = rng.standard_normal(bw.shape) + 1j * rng.standard_normal(bw.shape)
    bw = bw + sig / np.sqrt(2) * op.P[None] * noise
    L = np.linalg.cholesky(psi)
    braw = np.einsum("cd,dyx->cyx", L, bw)
    return maps, psi, mask, op, bw, braw


def _init_tv(lib, maps, psi, mask, braw, lam, T, inner, tile):
    ny, nx = maps.shape[1:]
    return lib.pico_init(ny, nx, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                         sampling=lib.PICO_CART_2D, recon=lib.PICO_CS_FISTA_TV,
                         kdata=_dev(braw.astype(np.complex64)), fista_iters=T,
                         cs_lambda=lam, tv_inner_iters=inner, probe_tile=tile)


@pytest.mark.parametrize("inner", [10, 7, 8, 3])
def test_tv_recon_jvp_and_noise_map_parity(lib, inner):
    say(f"case: TV-CS 64x96, 4 coils, Poisson-disc R=2 (8x8 calib), lam 1e-2, "
        f"FISTA 30, {inner} inner steps (multi-step passes{', one single step first' if inner % 2 else ''}, the last fused with the FISTA step); "
        f"3 JVPs, noise map of 6 probes in tiles 4+2")
    maps, psi, mask, op, bw, braw = _setup(64, 96, 4, 2.0, 8, seed=3)
    lam, T = 1e-2, 30
    h = _init_tv(lib, maps, psi, mask, braw, lam, T, inner, 4)
    xg = torch.empty((64, 96), dtype=torch.complex64, device="cuda:0")
    lib.pico_recon(h, xg)
    w = np.stack([ocs.kspace_probe(op, 8, i) for i in range(3)])
    ut = torch.empty((3, 64, 96), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_jvp(h, _dev(w.astype(np.complex64)), ut, 3)
    n = 64 * 96
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    lib.pico_noise_map(h, 21, 2, 6, 0, lib.make_accum(*acc_t))
    torch.cuda.synchronize()
    lib.pico_destroy(h)

    f = ocs.FistaTV(op, lam, T, inner)
    xr, zs = f.recon(bw, store=True)
    err = _rel(xg.cpu().numpy(), xr)
    say(f"  reconstruction rel err {err:.2e}")
    assert err < TOL
    u = ut.cpu().numpy()
    for k in range(3):
        e = _rel(u[k], f.jvp(w[k], zs))
        say(f"  jvp probe {k}: rel err {e:.2e}")
        assert e < TOL
    ref = ocs.noise_map_jvp(f, zs, 21, 2, 6)
    e = _rel(acc_t[0].cpu().numpy(), ref["sum"].ravel())
    say(f"  noise map (sum |J w|^2): rel err {e:.2e}")
    assert e < TOL


def test_tv_lambda_zero_equals_linear_map(lib):
    say("case: TV-CS with lam 0 (prox = identity, linear FISTA map): J w == recon of w; 96x64, 3 coils")
    maps, psi, mask, op, bw, braw = _setup(96, 64, 3, 2.0, 8, seed=4)
    h = _init_tv(lib, maps, psi, mask, braw, 0.0, 20, 5, 2)
    w = np.stack([ocs.kspace_probe(op, 1, i) for i in range(2)])
    ut = torch.empty((2, 96, 64), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_jvp(h, _dev(w.astype(np.complex64)), ut, 2)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    f = ocs.FistaTV(op, 0.0, 20, 5)
    for k in range(2):
        e = _rel(ut.cpu().numpy()[k], f.recon(w[k]))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL


def test_tv_single_inner_step_fully_sampled(lib):
    say("case: TV-CS 64x64, 2 coils, fully sampled, "
        "lam 5e-2, FISTA 12, 1 inner step; 2 JVPs")
    rng = np.random.default_rng(11)
    maps = workloads.coil_maps(64, 64, 2, rng)
    psi = workloads.noise_cov(2, rng)
    mask = np.ones((64, 64), np.uint8)
    op = opico.cartesian(maps, psi, mask)
    bw = op.forward(rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64)))
    braw = np.einsum("cd,dyx->cyx", np.linalg.cholesky(psi), bw)
    h = _init_tv(lib, maps, psi, mask, braw, 5e-2, 12, 1, 2)
    w = np.stack([ocs.kspace_probe(op, 3, i) for i in range(2)])
    ut = torch.empty((2, 64, 64), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_jvp(h, _dev(w.astype(np.complex64)), ut, 2)
    xg = torch.empty((64, 64), dtype=torch.complex64, device="cuda:0")
    lib.pico_recon(h, xg)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    f = ocs.FistaTV(op, 5e-2, 12, 1)
    xr, zs = f.recon(bw, store=True)
    e = _rel(xg.cpu().numpy(), xr)
    say(f"  reconstruction rel err {e:.2e}")
    assert e < TOL
    for k in range(2):
        e = _rel(ut.cpu().numpy()[k], f.jvp(w[k], zs))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL


def test_tv_pmr_parity(lib):
    say("case: TV-CS PMR 64x96, 3 coils, lam 1e-2, FISTA 15, 6 inner steps, sigma 0.02, "
        "10 replicas (FP64 replicas in batches of 4)")
    maps, psi, mask, op, bw, braw = _setup(64, 96, 3, 2.0, 8, seed=12)
    h = _init_tv(lib, maps, psi, mask, braw, 1e-2, 15, 6, 4)
    n = 64 * 96
    acc_t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    acc = lib.make_accum(*acc_t)
    lib.pico_pmr_cs(h, 5, 2, 10, 0.02, acc)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    f = ocs.FistaTV(op, 1e-2, 15, 6)
    ref = ocs.pmr_cs(f, bw, 5, 2, 10, 0.02)
    for key, t in zip(("sum", "sum_im", "sumsq"), acc_t):
        e = _rel(t.cpu().numpy(), ref[key].ravel())
        say(f"  {key}: rel err {e:.2e}")
        assert e < TOL


def test_tv_full_size_sampled_probes(lib):
    say("case: TV-CS 320x320, 15 coils, Poisson-disc R=2 (24x24 calib), lam 1e-2, FISTA 100, "
        "10 inner steps, K=64 tangents in one launch (63 zero probes); the last one checked")
    maps, psi, mask, op, bw, braw = _setup(320, 320, 15, 2.0, 24, seed=0)
    h = _init_tv(lib, maps, psi, mask, braw, 1e-2, 100, 10, 64)
    w = ocs.kspace_probe(op, 77, 63).astype(np.complex64)
    wt = torch.zeros((64, 15, 320, 320), dtype=torch.complex64, device="cuda:0")
    wt[63] = _dev(w)
    ut = torch.empty((64, 320, 320), dtype=torch.complex64, device="cuda:0")
    lib.pico_apply_jvp(h, wt, ut, 64)
    xg = torch.empty((320, 320), dtype=torch.complex64, device="cuda:0")
    lib.pico_recon(h, xg)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    f = ocs.FistaTV(op, 1e-2, 100, 10)
    xr, zs = f.recon(bw, store=True)
    e = _rel(xg.cpu().numpy(), xr)
    say(f"  reconstruction rel err {e:.2e}")
    assert e < TOL
    u = ut.cpu().numpy()
    assert float(np.abs(u[:63]).max()) == 0.0    # J is linear: zero probes give zero tangents
    e = _rel(u[63], f.jvp(w.astype(np.complex128), zs))
    say(f"  probe 63: rel err {e:.2e}")
    assert e < TOL
