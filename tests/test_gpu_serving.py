"""Serving loop on the GPU: device-byte accounting, results independent of
the mix (bit-identical to direct calls on fresh operators), FIFO admission
under an HBM budget, and one served request checked against the oracle."""
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


def _requests():
    """Small requests of every operator kind (kwargs of pico_init): phase-encode,
    2-D Cartesian, spiral with gridding, L1 and TV compressed sensing, and
    bfloat16 storage."""
    out = []
    rng = np.random.default_rng(21)
    maps = workloads.coil_maps(64, 64, 4, rng)
    out.append(("cart1d 64x64 4 coils R=2", dict(
        ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=workloads.noise_cov(4, rng),
        mask=_dev(workloads.cart_mask_1d(64, 2, 8)), cg_iters=20, probe_tile=8), 20))
    maps = workloads.coil_maps(64, 96, 5, rng)
    out.append(("cart2d 64x96 5 coils Tikhonov", dict(
        ny=64, nx=96, maps=_dev(maps.astype(np.complex64)), psi=workloads.noise_cov(5, rng),
        mask=_dev(workloads.poisson_disc_mask(64, 96, 2.0, 8, seed=5)), sampling=1, lam=0.05,
        cg_iters=15, probe_tile=6), 15))
    maps = workloads.coil_maps(64, 64, 4, rng)
    traj = workloads.spiral_traj(64, 2, 16, 512).astype(np.float32)
    out.append(("spiral 64x64 4 coils", dict(
        ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=workloads.noise_cov(4, rng),
        mask=None, sampling=2, lam=0.1, cg_iters=15, probe_tile=5, traj=_dev(traj),
        nsamples=traj.shape[0], oversamp=2.0, kb_width=6), 12))
    maps = workloads.coil_maps(64, 64, 3, rng)
    psi = workloads.noise_cov(3, rng)
    mask = workloads.poisson_disc_mask(64, 64, 2.0, 8, seed=6)
    x = workloads.phantom(64, rng)
    op = opico.cartesian(maps, psi, mask)
    b = op.forward(x)
    L = np.linalg.cholesky(psi)
    braw = np.einsum("cd,dyx->cyx", L, b).astype(np.complex64)
    out.append(("CS 64x64 3 coils", dict(
        ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=_dev(mask), sampling=1,
        recon=1, kdata=_dev(braw), fista_iters=20, cs_lambda=1e-3, wavelet_levels=3,
        probe_tile=4), 10))
    out.append(("TV-CS 64x64 3 coils", dict(
        ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=_dev(mask), sampling=1,
        recon=2, kdata=_dev(braw), fista_iters=12, cs_lambda=1e-2, tv_inner_iters=4,
        probe_tile=3), 7))
    maps = workloads.coil_maps(96, 64, 4, rng)
    out.append(("cart2d 96x64 4 coils, bfloat16 maps and planes", dict(
        ny=96, nx=64, maps=_dev(maps.astype(np.complex64)), psi=workloads.noise_cov(4, rng),
        mask=_dev(workloads.poisson_disc_mask(96, 64, 2.0, 8, seed=7)), sampling=1, cg_iters=12,
        probe_tile=4, storage=2), 9))
    return out


def _acc(n):
    t = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    return t


def _direct(lib, kw, seed, nprobes):
    kw = dict(kw)
    ny, nx = kw.pop("ny"), kw.pop("nx")
    maps, psi, mask = kw.pop("maps"), kw.pop("psi"), kw.pop("mask")
    h = lib.pico_init(ny, nx, maps, psi, mask, **kw)
    t = _acc(ny * nx)
    acc = lib.make_accum(*t)
    lib.pico_noise_map(h, seed, 0, nprobes, 0, acc)
    torch.cuda.synchronize()
    by = lib.pico_op_bytes(h)
    lib.pico_destroy(h)
    return t, by


def _serve(lib, reqs, budget, slots, depth, seed=17):
    srv = lib.Server(budget, slots, depth)
    accs = []
    ids = []
    for name, kw, nprobes in reqs:
        accs.append(_acc(kw["ny"] * kw["nx"]))
    torch.cuda.synchronize()        # the server's streams do not wait on torch's stream
    for (name, kw, nprobes), t in zip(reqs, accs):
        ids.append(srv.submit(seed, 0, nprobes, lib.make_accum(*t), **kw))
    srv.wait_idle(120.0)
    info = {r["id"]: r for r in srv.poll()}
    srv.close()
    torch.cuda.synchronize()
    return accs, [info[i] for i in ids]


def test_estimate_matches_actual_bytes(lib):
    for name, kw, _ in _requests():
        say(f"case: bytes of {name}")
        d, keep = lib.make_desc(**kw)
        est = lib.pico_estimate_bytes(d)
        _, act = _direct(lib, kw, 1, 1)
        say(f"  estimate {est}  actual {act}")
        assert est == act


def test_served_results_equal_direct_calls(lib):
    reqs = _requests()
    direct = [_direct(lib, kw, 17, n)[0] for _, kw, n in reqs]
    for slots, depth in ((1, 1), (4, 2), (3, 3)):
        say(f"case: mix of {len(reqs)} requests, {slots} slots, {depth} tiles in flight, budget 4 GiB")
        accs, info = _serve(lib, reqs, 4 << 30, slots, depth)
        for (name, _, n), d, a, r in zip(reqs, direct, accs, info):
            assert r["status"] == 0, r["error"]
            assert r["probes"] == n
            for x, y in zip(d, a):
                assert torch.equal(x, y), name
        say("  bit-identical to direct calls")


def test_budget_admission_is_fifo_and_exclusive(lib):
    reqs = _requests()
    peaks = []
    for _, kw, _ in reqs:
        d, keep = lib.make_desc(**kw)
        peaks.append(lib.pico_estimate_bytes(d)[1])
    budget = int(max(peaks) * 1.05)
    say(f"case: budget {budget} B (1.05 x the largest peak), 4 slots, 2 tiles in flight")
    accs, info = _serve(lib, reqs, budget, 4, 2)
    assert all(r["status"] == 0 for r in info)
    order = sorted(info, key=lambda r: r["t_admit_ms"])
    assert [r["id"] for r in order] == [r["id"] for r in info]       # arrival order
    for r in info:
        assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]
    direct = [_direct(lib, kw, 17, n)[0] for _, kw, n in reqs]
    for d, a in zip(direct, accs):
        for x, y in zip(d, a):
            assert torch.equal(x, y)
    srv = lib.Server(budget // 4, 2, 2)
    big = max(range(len(reqs)), key=lambda i: peaks[i])
    with pytest.raises(lib.PicoError) as ei:
        srv.submit(1, 0, 4, lib.make_accum(*_acc(64 * 64)), **reqs[big][1])
    assert ei.value.status == lib.PICO_ENOMEM
    srv.close()


def test_served_request_matches_oracle(lib):
    say("case: served cart1d 64x64 request (20 probes, tiles of 8) vs the FP64 oracle")
    rng = np.random.default_rng(31)
    maps = workloads.coil_maps(64, 64, 4, rng)
    psi = workloads.noise_cov(4, rng)
    mask = workloads.cart_mask_1d(64, 2, 8)
    kw = dict(ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi, mask=_dev(mask),
              cg_iters=20, probe_tile=8)
    accs, info = _serve(lib, [("cart1d", kw, 20)], 1 << 30, 2, 2, seed=5)
    assert info[0]["status"] == 0
    ref = opico.noise_map(opico.Covariance(opico.cartesian(maps, psi, mask), 0.0, 20), 5, 0, 20)
    got = accs[0][0].cpu().numpy()
    e = float(np.linalg.norm(got - ref["sum"].ravel()) / np.linalg.norm(ref["sum"]))
    say(f"  rel err {e:.2e}")
    assert e < 1e-4


def _serve_seq(lib, srv, reqs, seed=17):
    """Submit requests one after the other (each waits for the previous)."""
    accs, info = [], []
    for name, kw, nprobes in reqs:
        t = _acc(kw["ny"] * kw["nx"])
        torch.cuda.synchronize()
        rid = srv.submit(seed, 0, nprobes, lib.make_accum(*t), **kw)
        srv.wait_idle(120.0)
        info += [r for r in srv.poll() if r["id"] == rid]
        accs.append(t)
    torch.cuda.synchronize()
    return accs, info


def test_resident_operators_are_reused_by_content(lib):
    reqs = _requests()
    name, kw, n = reqs[0]
    kw = dict(kw, graph=1)
    say(f"case: {name} served 3 times on one resident operator, then with changed map contents")
    srv = lib.Server(4 << 30, 2, 2)
    accs, info = _serve_seq(lib, srv, [(name, kw, n)] * 3)
    assert [r["op_reused"] for r in info] == [0, 1, 1]
    st = srv.cache_stats()
    assert st["hits"] == 2 and st["misses"] == 1 and st["resident_ops"] == 1
    d, _ = _direct(lib, kw, 17, n)
    for a in accs:
        for x, y in zip(d, a):
            assert torch.equal(x, y)
    # same device pointer, different contents: a different key, a new operator
    kw["maps"].mul_(1.25)
    torch.cuda.synchronize()
    accs2, info2 = _serve_seq(lib, srv, [(name, kw, n)])
    assert info2[0]["op_reused"] == 0 and srv.cache_stats()["resident_ops"] == 2
    d2, _ = _direct(lib, kw, 17, n)
    for x, y in zip(d2, accs2[0]):
        assert torch.equal(x, y)
    assert not torch.equal(d2[0], d[0])
    kw["maps"].div_(1.25)
    srv.close()


def test_idle_operators_are_evicted_for_room(lib):
    reqs = _requests()[:3]
    peaks = []
    for _, kw, _ in reqs:
        d, keep = lib.make_desc(**kw)
        peaks.append(lib.pico_estimate_bytes(d)[1])
    budget = int(max(peaks) * 1.05)
    say(f"case: 3 kinds in a budget of 1.05 x the largest peak ({budget} B), served in turn twice")
    srv = lib.Server(budget, 1, 2)
    accs, info = _serve_seq(lib, srv, reqs + reqs)
    assert all(r["status"] == 0 for r in info)
    st = srv.cache_stats()
    assert st["resident_ops"] >= 1 and st["resident_bytes"] <= budget
    srv.close()
    for (name, kw, n), a in zip(reqs + reqs, accs):
        d, _ = _direct(lib, kw, 17, n)
        for x, y in zip(d, a):
            assert torch.equal(x, y), name


def test_autotune_and_auto_tile_requests(lib, tmp_path):
    rng = np.random.default_rng(41)
    maps = workloads.coil_maps(64, 64, 4, rng)
    psi = workloads.noise_cov(4, rng)
    kw = dict(ny=64, nx=64, maps=_dev(maps.astype(np.complex64)), psi=psi,
              mask=_dev(workloads.cart_mask_1d(64, 2, 8)), cg_iters=20, probe_tile=0)
    cache = str(tmp_path / "tune.txt")
    say("case: autotune a 64x64 4-coil phase-encode operator (tiles 16..512, three normal forms, graph "
        "or not), then a served request with probe_tile 0 takes the cached shape")
    d, keep = lib.make_desc(**dict(kw, probe_tile=1))
    t1 = lib.pico_autotune(d, 1 << 30, cache)
    say(f"  tuned: {t1}")
    assert not t1["from_cache"] and t1["probe_tile"] in (16, 32, 64, 128, 256, 512)
    assert t1["normal_form"] in (1, 2, 3) and t1["probes_per_s"] > 0
    t2 = lib.pico_autotune(d, 1 << 30, cache)
    assert t2["from_cache"] and t2["probe_tile"] == t1["probe_tile"]
    srv = lib.Server(2 << 30, 2, 2)
    accs, info = _serve_seq(lib, srv, [("auto, untuned", kw, 40)])
    assert info[0]["probe_tile"] == 64 and info[0]["status"] == 0     # size rule: 256 at 64^2, cut to < 2 x 40 probes
    srv.set_tuning(cache)
    accs, info = _serve_seq(lib, srv, [("auto, tuned", kw, 40)])
    assert info[0]["probe_tile"] == t1["probe_tile"] and info[0]["status"] == 0
    srv.close()
    dk = dict(kw, probe_tile=t1["probe_tile"], normal_form=t1["normal_form"], graph=t1["graph"])
    ref, _ = _direct(lib, dk, 17, 40)
    for x, y in zip(ref, accs[0]):
        assert torch.equal(x, y)
