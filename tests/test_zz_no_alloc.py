"""pico_pmr_cs_noalloc (replica workspace in the library's static device
array) against pico_pmr_cs (workspace allocated on its first call): the same
sums, on two calls in a row, the second on a smaller operator; an operator
whose replica workspace exceeds the static array is refused."""
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


def _cs_op(lib, n, nc, recon, tile, T, seed):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n, n, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    x = workloads.phantom(n, rng)
    mask = workloads.poisson_disc_mask(n, n, 2.0, 8, seed=seed)
    op = opico.cartesian(maps, psi, mask)
    bw = op.forward(x)
    bw = bw + 1e-3 * op.P[None] * (rng.standard_normal(bw.shape) + 1j * rng.standard_normal(bw.shape))
    braw = np.einsum("cd,dyx->cyx", np.linalg.cholesky(psi), bw)
    return lib.pico_init(n, n, _dev(maps.astype(np.complex64)), psi, _dev(mask),
                         sampling=lib.PICO_CART_2D, recon=recon, kdata=_dev(braw.astype(np.complex64)),
                         fista_iters=T, cs_lambda=1e-3, wavelet_levels=2, probe_tile=tile, tv_inner_iters=4)


def _accs(n):
    return [torch.zeros(n * n, dtype=torch.float64, device="cuda:0") for _ in range(3)]


def _run(lib, h, n, fn, nrep):
    s = _accs(n)
    acc = lib.make_accum(*s)
    fn(h, 5, 3, nrep, 0.02, acc)
    torch.cuda.synchronize()
    assert acc.count == nrep
    return [t.cpu().numpy() for t in s]


def test_noalloc_matches_pmr_cs_on_two_calls(lib):
    cases = [(96, 4, lib.PICO_CS_FISTA_L1WAV, 4, 6), (64, 2, lib.PICO_CS_FISTA_TV, 3, 5)]
    for n, nc, recon, tile, nrep in cases:
        say(f"case: pico_pmr_cs_noalloc vs pico_pmr_cs, {n}x{n}, {nc} coils, recon {recon}, "
            f"tile {tile}, {nrep} replicas")
        h = _cs_op(lib, n, nc, recon, tile, 12, seed=n)
        got = _run(lib, h, n, lib.pico_pmr_cs_noalloc, nrep)
        ref = _run(lib, h, n, lib.pico_pmr_cs, nrep)
        for g, r in zip(got, ref):
            assert np.all(np.isfinite(g))
            assert np.linalg.norm(g - r) <= 1e-12 * np.linalg.norm(r)
            assert np.array_equal(g, r)       # same kernels, same batches: bitwise
        lib.pico_destroy(h)


def test_noalloc_refuses_workspace_beyond_the_static_array(lib):
    say("case: pico_pmr_cs_noalloc on 128x128, 8 coils, tile 16 (92 MB > 64 MiB) -> PICO_EINVAL")
    h = _cs_op(lib, 128, 8, lib.PICO_CS_FISTA_L1WAV, 16, 2, seed=7)
    s = _accs(128)
    acc = lib.make_accum(*s)
    with pytest.raises(lib.PicoError) as ei:
        lib.pico_pmr_cs_noalloc(h, 5, 0, 4, 0.02, acc)
    assert ei.value.status == lib.PICO_EINVAL
    assert "64 MiB" in str(ei.value) and acc.count == 0
    lib.pico_destroy(h)
