"""Host-side pieces of the serving loop: the arena's offset bookkeeping
(compiled with g++ against the library's own header) and the device-byte
estimate pico_init's admission uses (no GPU needed)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_09590_amd", "csrc")


# the second build runs the same checks under AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; any report fails the run)
SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.parametrize("flags", [[], SANITIZE], ids=["plain", "asan_ubsan"])
def test_arena_bookkeeping(tmp_path, flags):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "arena_check")
    subprocess.run([gxx, "-std=c++17", "-O1", *flags, "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "arena_check.cpp"), "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout


@pytest.fixture(scope="module")
def p():
    from paper_2605_09590_amd import pico as p
    p.load()
    return p


def _round(b):
    return (max(b, 1) + 255) // 256 * 256


def test_estimate_cart1d_closed_form(p):
    n, K, nc = 320 * 320, 256, 15
    expect = (_round(n * nc * 8) + 4 * _round(n * K * 8) + _round(K * 320 * 4 * 8) + _round(512 * 8)
              + 4 * _round(K * 8) + _round(K * 4) + _round(320 * 4) + _round(320 * 8))
    d, _ = p.make_desc(320, 320, 0x1000, None, 0x2000, ncoils=15, probe_tile=256, cg_iters=30,
                       normal_form=1)
    res, peak = p.pico_estimate_bytes(d)
    assert res == expect
    assert peak == expect + _round(2 * nc * nc * 8)      # the whitening matrix during init
    # dense form: + the 320 blocks of 320 x 320 complex64 and the circulant
    d, _ = p.make_desc(320, 320, 0x1000, None, 0x2000, ncoils=15, probe_tile=256, cg_iters=30,
                       normal_form=2)
    res, peak = p.pico_estimate_bytes(d)
    assert res == expect + _round(320 * 320 * 320 * 8) + _round(320 * 16)
    # split-FP16 dense form: the same blocks as FP16 pairs, plus the column
    # and per-tile probe exponents
    d, _ = p.make_desc(320, 320, 0x1000, None, 0x2000, ncoils=15, probe_tile=256, cg_iters=30,
                       normal_form=3)
    res, _ = p.pico_estimate_bytes(d)
    assert res == (expect + _round(320 * 320 * 320 * 8) + _round(320 * 16) + _round(320 * 4)
                   + _round(320 * 8 * 32 * 4))
    d, _ = p.make_desc(320, 320, 0x1000, None, 0x2000, ncoils=15, probe_tile=256, cg_iters=30)
    assert p.pico_estimate_bytes(d)[0] == expect         # the default is the FFT form


def test_estimate_grows_with_tile_and_kind(p):
    base, _ = p.make_desc(128, 128, 0x1000, None, 0x2000, ncoils=8, probe_tile=16,
                          sampling=p.PICO_CART_2D)
    r1, _ = p.pico_estimate_bytes(base)
    big, _ = p.make_desc(128, 128, 0x1000, None, 0x2000, ncoils=8, probe_tile=32,
                         sampling=p.PICO_CART_2D)
    r2, _ = p.pico_estimate_bytes(big)
    assert r2 > r1
    cs, _ = p.make_desc(128, 128, 0x1000, None, 0x2000, ncoils=8, probe_tile=16,
                        sampling=p.PICO_CART_2D, recon=p.PICO_CS_FISTA_L1WAV, kdata=0x3000,
                        fista_iters=100, wavelet_levels=4)
    rc, pc = p.pico_estimate_bytes(cs)
    assert rc >= r1 + 100 * 128 * 128 * 16       # the stored FP64 coefficients
    assert pc > rc                               # FP64 primal temporaries
    sp, _ = p.make_desc(128, 128, 0x1000, None, None, ncoils=8, probe_tile=16,
                        sampling=p.PICO_NONCART, traj=0x4000, nsamples=50000, lam=0.1)
    rs, ps = p.pico_estimate_bytes(sp)
    assert ps > rs                               # Toeplitz build scratch
    kb, _ = p.make_desc(128, 128, 0x1000, None, None, ncoils=8, probe_tile=16,
                        sampling=p.PICO_NONCART, traj=0x4000, nsamples=50000, lam=0.1,
                        oversamp=2.0, kb_width=6)
    rk, _ = p.pico_estimate_bytes(kb)
    # gridding tables in bin order: 2 tap starts + 2 x 6 weights + the sample
    # index per sample, and the [K][256][256] grid
    assert rk - rs >= 50000 * (8 + 48 + 4) + 16 * 256 * 256 * 8
    # the gridding normal operator: a second [K][256][256] grid and the stencil
    # ((2W - 1)^2 weights per grid point) in place of the Toeplitz kernels
    kbn, _ = p.make_desc(128, 128, 0x1000, None, None, ncoils=8, probe_tile=16,
                         sampling=p.PICO_NONCART, traj=0x4000, nsamples=50000, lam=0.1,
                         oversamp=2.0, kb_width=6, noncart_normal=1)
    rn, pn = p.pico_estimate_bytes(kbn)
    grid2_and_stencil = 16 * 256 * 256 * 8 + 256 * 256 * 121 * 4
    assert rn >= 50000 * (8 + 48 + 4) + 16 * 256 * 256 * 8 + grid2_and_stencil
    assert rn - rk < grid2_and_stencil           # no Toeplitz kernels held
    bad, _ = p.make_desc(128, 128, 0x1000, None, None, ncoils=8, probe_tile=16,
                         sampling=p.PICO_NONCART, traj=0x4000, nsamples=50000, oversamp=1.1,
                         kb_width=6)
    with pytest.raises(p.PicoError):
        p.pico_estimate_bytes(bad)               # 1.1 * 128 is not an integer


def test_estimate_validates(p):
    d, _ = p.make_desc(63, 64, 0x1000, None, 0x2000, ncoils=4)
    with pytest.raises(p.PicoError) as ei:
        p.pico_estimate_bytes(d)
    assert ei.value.status == p.PICO_EINVAL


def test_estimate_validates_normal_form(p):
    # the dense forms need a phase-encode mask and ny a multiple of 32 in 64..512
    ok, _ = p.make_desc(96, 40, 0x1000, None, 0x2000, ncoils=4, normal_form=3)
    p.pico_estimate_bytes(ok)
    for form in (2, 3):
        for ny in (100, 32, 544):
            d, _ = p.make_desc(ny, 40, 0x1000, None, 0x2000, ncoils=4, normal_form=form)
            with pytest.raises(p.PicoError) as ei:
                p.pico_estimate_bytes(d)
            assert ei.value.status == p.PICO_EINVAL
        d, _ = p.make_desc(96, 40, 0x1000, None, 0x2000, ncoils=4, sampling=p.PICO_CART_2D, normal_form=form)
        with pytest.raises(p.PicoError) as ei:
            p.pico_estimate_bytes(d)
        assert ei.value.status == p.PICO_EINVAL
    for bad in (-1, 4):
        d, _ = p.make_desc(96, 40, 0x1000, None, 0x2000, ncoils=4, normal_form=bad)
        with pytest.raises(p.PicoError) as ei:
            p.pico_estimate_bytes(d)
        assert ei.value.status == p.PICO_EINVAL


def test_estimate_tv_counts_projection_data(p):
    kw = dict(ncoils=8, probe_tile=16, sampling=p.PICO_CART_2D, recon=p.PICO_CS_FISTA_TV, kdata=0x3000,
              fista_iters=50)
    d10, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, tv_inner_iters=10, **kw)
    d20, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, tv_inner_iters=20, **kw)
    r10, p10 = p.pico_estimate_bytes(d10)
    r20, _ = p.pico_estimate_bytes(d20)
    # 20 bytes (w^ as 2 complex64 and 1/|w| as float32) per pixel per inner step
    assert r20 - r10 == _round(50 * 20 * 128 * 96 * 16) + _round(50 * 20 * 128 * 96 * 4) \
        - _round(50 * 10 * 128 * 96 * 16) - _round(50 * 10 * 128 * 96 * 4)
    assert p10 > r10                             # FP64 primal and dual temporaries
    for bad in (0, 1001):
        d, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, tv_inner_iters=bad, **kw)
        with pytest.raises(p.PicoError) as ei:
            p.pico_estimate_bytes(d)
        assert ei.value.status == p.PICO_EINVAL


def test_estimate_counts_bf16_maps(p):
    base = dict(ncoils=8, probe_tile=16, sampling=p.PICO_CART_2D)
    d0, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, **base)
    r0, _ = p.pico_estimate_bytes(d0)
    for st in (p.PICO_BF16_MAPS, p.PICO_BF16_STREAM):
        d, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, storage=st, **base)
        assert p.pico_estimate_bytes(d)[0] == r0 + _round(8 * 128 * 96 * 4)   # packed bfloat16 maps
    d, _ = p.make_desc(128, 96, 0x1000, None, 0x2000, storage=3, **base)
    with pytest.raises(p.PicoError) as ei:
        p.pico_estimate_bytes(d)
    assert ei.value.status == p.PICO_EINVAL
