"""Edge cases on the GPU: empty probe ranges, single-probe tiles, the largest
built transform lengths, a one-line mask under Tikhonov, an empty mask (CG breakdown reported,
never a hang), and argument errors that must leave the accumulators alone.
Parity against the FP64 oracle where a result is defined."""
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


def _acc(n, k=3):
    t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(k)]
    return t


def test_empty_range_and_single_probe_tiles(lib):
    say("case: 0 probes (no-op), then 3 probes in tiles of 1, 64x32 3 coils")
    prob = workloads.config(2, seed=6, ny=64, nx=32, nc=3, acs=8, cg_iters=15)
    h = lib.pico_init(64, 32, _dev(prob.maps.astype(np.complex64)), prob.psi, _dev(prob.mask),
                      cg_iters=15, probe_tile=1)
    t = _acc(64 * 32)
    acc = lib.make_accum(*t)
    lib.pico_noise_map(h, 4, 0, 0, 0, acc)
    torch.cuda.synchronize()
    assert acc.count == 0 and all(float(x.abs().max()) == 0.0 for x in t)
    lib.pico_noise_map(h, 4, 0, 3, 0, acc)
    torch.cuda.synchronize()
    # argument errors leave the accumulators untouched
    before = [x.clone() for x in t]
    with pytest.raises(lib.PicoError):
        lib.pico_noise_map(h, 4, -1, 3, 0, acc)
    with pytest.raises(lib.PicoError):
        lib.pico_noise_map(h, 4, 0, 3, 9, acc)
    torch.cuda.synchronize()
    assert acc.count == 3 and all(torch.equal(a, b) for a, b in zip(before, t))
    lib.pico_destroy(h)
    ref = opico.noise_map(opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 15), 4, 0, 3)
    e = _rel(t[0].cpu().numpy(), ref["sum"].ravel())
    say(f"  rel err {e:.2e}")
    assert e < TOL


@pytest.mark.parametrize("form", [0, 3])
def test_largest_phase_encode_length(lib, form):
    say(f"case: phase-encode 512x512 (largest column FFT, largest dense block), 2 coils R=2 + 24 ACS, "
        f"4 probes, CG 20, normal form {form}")
    prob = workloads.config(2, seed=7, ny=512, nx=512, nc=2, acs=24, cg_iters=20)
    h = lib.pico_init(512, 512, _dev(prob.maps.astype(np.complex64)), prob.psi, _dev(prob.mask),
                      cg_iters=20, probe_tile=4, normal_form=form)
    t = _acc(512 * 512)
    lib.pico_noise_map(h, 8, 0, 4, 0, lib.make_accum(*t))
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    ref = opico.noise_map(opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, 20), 8, 0, 4)
    e = _rel(t[0].cpu().numpy(), ref["sum"].ravel())
    say(f"  rel err {e:.2e}")
    assert e < TOL


def test_largest_grid_length_spiral(lib):
    say("case: spiral 384x384 (Toeplitz grid 768, the largest FFT), 2 coils, 12x1024 R=1, "
        "lambda 0.1, apply_cov on 1 probe, CG 15")
    rng = np.random.default_rng(2)
    maps = workloads.coil_maps(384, 384, 2, rng)
    psi = workloads.noise_cov(2, rng)
    traj = workloads.spiral_traj(384, 1, 12, 1024).astype(np.float32)
    h = lib.pico_init(384, 384, _dev(maps.astype(np.complex64)), psi, None, sampling=lib.PICO_NONCART,
                      lam=0.1, cg_iters=15, probe_tile=1, traj=_dev(traj), nsamples=traj.shape[0])
    v = (rng.standard_normal((1, 384, 384)) + 1j * rng.standard_normal((1, 384, 384)))
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 1)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    op = onufft.NonCartOp(maps, psi, traj.astype(np.float64))
    ref = opico.Covariance(op, 0.1, 15).apply(v[0])
    e = _rel(ut.cpu().numpy()[0], ref)
    say(f"  rel err {e:.2e}")
    assert e < TOL


def test_single_line_mask_with_tikhonov(lib):
    say("case: one sampled line of 64 (M rank one per column), lambda 0.2: Sigma stays defined; "
        "apply_cov on 2 probes, CG 25")
    rng = np.random.default_rng(3)
    maps = workloads.coil_maps(64, 16, 2, rng)
    psi = workloads.noise_cov(2, rng)
    mask = np.zeros(64, np.uint8)
    mask[32] = 1
    h = lib.pico_init(64, 16, _dev(maps.astype(np.complex64)), psi, _dev(mask), lam=0.2, cg_iters=25,
                      probe_tile=2)
    v = rng.standard_normal((2, 64, 16)) + 1j * rng.standard_normal((2, 64, 16))
    vt = _dev(v.astype(np.complex64))
    ut = torch.empty_like(vt)
    lib.pico_apply_cov(h, vt, ut, 2)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    cov = opico.Covariance(opico.cartesian(maps, psi, mask), 0.2, 25)
    for k in range(2):
        e = _rel(ut.cpu().numpy()[k], cov.apply(v[k]))
        say(f"  probe {k}: rel err {e:.2e}")
        assert e < TOL


@pytest.mark.parametrize("form", [0, 2, 3])
def test_empty_mask_reports_breakdown(lib, form):
    say(f"case: no sampled line (M = 0), lambda 0: every CG right-hand side breaks down at once; "
        f"PICO_ENOTCONV with all probes frozen, the map written as zeros; normal form {form} "
        f"(dense blocks of zeros)")
    rng = np.random.default_rng(4)
    maps = workloads.coil_maps(64, 16, 1, rng)
    h = lib.pico_init(64, 16, _dev(maps.astype(np.complex64)), None, _dev(np.zeros(64, np.uint8)),
                      cg_iters=10, probe_tile=4, normal_form=form)
    t = _acc(64 * 16)
    st = lib.pico_stats_t()
    with pytest.raises(lib.PicoError) as ei:
        lib.pico_noise_map(h, 1, 0, 4, 0, lib.make_accum(*t), st)
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    say(f"  status {ei.value.status}, frozen {st.frozen} of {st.probes}")
    assert ei.value.status == lib.PICO_ENOTCONV and st.frozen == 4 and st.probes == 4
    assert float(t[0].abs().max()) == 0.0
