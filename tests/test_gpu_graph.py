"""Probe tiles replayed from HIP graphs (pico_op_desc_t.graph = 1) against
direct launches of the same operator description: every replay's
accumulators must be bitwise those of the direct path, with eager work and
synchronisations between the replays, for every operator kind; a new
accumulator triggers a new capture; ragged last tiles get their own graph.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import pico as opico

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def _cart1d(lib, n=64, nc=4, lam=0.0, form=0):
    prob = workloads.config(1, seed=2, ny=n, nx=n, nc=nc) if n != 64 else workloads.config(1, seed=2)
    return dict(ny=prob.ny, nx=prob.nx, maps=_dev(prob.maps.astype(np.complex64)), psi=prob.psi,
                mask=_dev(prob.mask), cg_iters=12, lam=lam, normal_form=form)


def _cart2d(lib, lam=0.05):
    rng = np.random.default_rng(3)
    maps = workloads.coil_maps(64, 96, 3, rng)
    psi = workloads.noise_cov(3, rng)
    mask = workloads.poisson_disc_mask(64, 96, 2.0, 8, seed=3)
    return dict(ny=64, nx=96, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=_dev(mask),
                sampling=lib.PICO_CART_2D, cg_iters=10, lam=lam)


def _spiral(lib):
    rng = np.random.default_rng(4)
    maps = workloads.coil_maps(64, 64, 4, rng)
    psi = workloads.noise_cov(4, rng)
    traj = workloads.spiral_traj(64, R=2, interleaves=16, samples=512).astype(np.float32)
    return dict(ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=None,
                sampling=lib.PICO_NONCART, traj=_dev(traj), nsamples=traj.shape[0], lam=0.1, cg_iters=10)


def _cs(lib, tv):
    rng = np.random.default_rng(5)
    maps = workloads.coil_maps(64, 64, 3, rng)
    psi = workloads.noise_cov(3, rng)
    x = workloads.phantom(64, rng)
    mask = workloads.poisson_disc_mask(64, 64, 2.0, 8, seed=5)
    op = opico.cartesian(maps, psi, mask)
    bw = op.forward(x)
    braw = np.einsum("cd,dyx->cyx", np.linalg.cholesky(psi), bw)
    return dict(ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=_dev(mask),
                sampling=lib.PICO_CART_2D, recon=lib.PICO_CS_FISTA_TV if tv else lib.PICO_CS_FISTA_L1WAV,
                kdata=_dev(braw.astype(np.complex64)), fista_iters=15, cs_lambda=1e-2 if tv else 1e-3,
                wavelet_levels=3, tv_inner_iters=4)


CASES = {
    "cart1d_fft": lambda lib: _cart1d(lib),
    "cart1d_fft_tikhonov": lambda lib: _cart1d(lib, lam=0.1),
    "cart1d_split_fp16": lambda lib: _cart1d(lib, form=3),
    "cart2d_tikhonov": _cart2d,
    "spiral_toeplitz": _spiral,
    "cs_l1": lambda lib: _cs(lib, False),
    "cs_tv": lambda lib: _cs(lib, True),
}


def _accs(n):
    return [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]


@pytest.mark.parametrize("kind", list(CASES))
def test_graph_replays_match_direct_launches(lib, kind):
    kw = CASES[kind](lib)
    tile = 5
    say(f"case: graph replay vs direct, {kind}, {kw['ny']}x{kw['nx']}, tile {tile}, "
        "4 calls of 12 probes (2 full tiles + a ragged 2 each)")
    n = kw["ny"] * kw["nx"]
    hd = lib.pico_init(probe_tile=tile, graph=0, **kw)
    hg = lib.pico_init(probe_tile=tile, graph=1, **kw)
    ad, ag = _accs(n), _accs(n)
    acc_d, acc_g = lib.make_accum(*ad), lib.make_accum(*ag)
    for call in range(4):
        first = 12 * call + 3
        lib.pico_noise_map(hg, 77, first, 12, call % 2 * 2, acc_g)      # families 0 and 2
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda:0") * 2.0                  # eager work between replays
        lib.pico_noise_map(hd, 77, first, 12, call % 2 * 2, acc_d)
        torch.cuda.synchronize()
        del junk
        for a, b in zip(ag, ad):
            assert torch.equal(a, b), (kind, call)
        assert acc_g.count == acc_d.count == 12 * (call + 1)
    # a second accumulator on the same operator: a new capture, same values
    ag2 = _accs(n)
    acc2 = lib.make_accum(*ag2)
    lib.pico_noise_map(hg, 77, 3, 12, 0, acc2)
    ad2 = _accs(n)
    lib.pico_noise_map(hd, 77, 3, 12, 0, lib.make_accum(*ad2))
    torch.cuda.synchronize()
    for a, b in zip(ag2, ad2):
        assert torch.equal(a, b)
    lib.pico_destroy(hg)
    lib.pico_destroy(hd)


def test_graph_full_size_headline_tile(lib):
    say("case: graph replay vs direct, 320x320 15 coils R=2+24 ACS, K=256, CG 30, 3 tiles")
    prob = workloads.config(2, seed=0)
    kw = dict(ny=320, nx=320, maps=_dev(prob.maps.astype(np.complex64)), psi=prob.psi,
              mask=_dev(prob.mask), cg_iters=30)
    n = 320 * 320
    hd = lib.pico_init(probe_tile=256, graph=0, **kw)
    hg = lib.pico_init(probe_tile=256, graph=1, **kw)
    ad, ag = _accs(n), _accs(n)
    acc_d, acc_g = lib.make_accum(*ad), lib.make_accum(*ag)
    for t in range(3):
        lib.pico_noise_map(hg, 5, 256 * t, 256, 0, acc_g)
        lib.pico_noise_map(hd, 5, 256 * t, 256, 0, acc_d)
        torch.cuda.synchronize()
        for a, b in zip(ag, ad):
            assert torch.equal(a, b), t
    lib.pico_destroy(hg)
    lib.pico_destroy(hd)
