#!/usr/bin/env python3
"""Benchmark of the PICO noise-map hot path on one MI355X.

Workload: 2-D Cartesian SENSE, 320 x 320 complex64 image, 15 coils with
synthetic Gaussian-profile sensitivities, random SPD channel covariance,
R=2 uniform phase-encode undersampling plus 24 fully sampled centre lines,
K=256 random-phase probes solved as one batched CG of 30 iterations with
FP64 inner products and accumulators.

One step = one pico_noise_map call over 256 probes: probe generation, the
256 CG solves and the FP64 accumulation, with all inputs resident in HBM.
Printed: one JSON line (throughput in probe-solves/s, time to a 1 % NRMSE
standard-deviation map against the exact map, roofline of the dominant
kernel measured with HIP events, the FP64 CPU oracle timed on a bounded
sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1%-error noise map (s) + probe solves/s; p50/p99 request latency"
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("cart1d_normal.h", "fft.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2605_09590_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def gram16_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("gram.hip", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2605_09590_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def normal_op_flops(ny, nx, nc):
    """Algorithmic FLOPs of one application of M to one probe (separable path).

    Per coil and image column: two length-ny FFTs at 5 n log2 n, the map
    product (6 n), the mask weight (2 n) and the conjugate map product with
    accumulation (8 n).
    """
    n = ny
    per_line = 2 * 5 * n * math.log2(n) + 16 * n
    return nc * nx * per_line


def cs_kspace_arrays(torch, dev, maps, psi, mask, x, snr_db, seed=0):
    """Raw multi-coil k-space b = P F_c (S x) + L n, formed on the GPU with
    torch.fft (input synthesis, outside every timed region): phantom x, raw maps
    S, centred orthonormal 2-D DFT F_c, noise with covariance Psi = L L^H at the
    given input SNR over the sampled locations."""
    import numpy as np
    x = torch.from_numpy(x.astype(np.complex128)).to(dev)
    maps = torch.from_numpy(maps.astype(np.complex128)).to(dev)
    mask = torch.from_numpy(mask.astype(np.float64)).to(dev)
    img = maps * x[None]
    k = torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(img, dim=(-2, -1)), norm="ortho"),
                           dim=(-2, -1)) * mask[None]
    sig = torch.sqrt(torch.mean(torch.abs(k[:, mask > 0]) ** 2)) * 10 ** (-snr_db / 20)
    rng = np.random.default_rng(seed + 1000)
    nz = rng.standard_normal(k.shape) + 1j * rng.standard_normal(k.shape)
    L = torch.from_numpy(np.linalg.cholesky(psi)).to(dev)
    n = torch.einsum("cd,dyx->cyx", L, torch.from_numpy(nz).to(dev)) * (sig / math.sqrt(2.0))
    return (k + n * mask[None]).to(torch.complex64).contiguous()


def cs_kspace(torch, dev, prob, seed=0):
    """k-space data of the CS workload (phantom, maps, Psi, mask of ``prob``)."""
    return cs_kspace_arrays(torch, dev, prob.maps, prob.psi, prob.mask, prob.extra["phantom"],
                            prob.extra["snr_db"], seed)


def serve_pool(workloads, torch, np, dev, n_ops, sizes, coils, seed=0):
    """Seeded pool of distinct operators (protocols) for the serving workload:
    kind Cartesian (phase-encode R=2 + 24 ACS, CG 30) / spiral (48x4096
    interleaves at R=2, lambda 0.1, CG 30) / CS (Poisson-disc R=2 + 24x24
    calibration, FISTA 100, lambda 1e-3, 4 db4 levels) with probabilities
    0.4 / 0.4 / 0.2, matrix size from ``sizes``, coils uniform in ``coils``;
    the first operator is forced to the largest size and coil count, the second
    to the smallest, so the pool spans the ranges.  probe_tile 0 (the server
    takes the tuned tile), graph replay on; device inputs resident."""
    rng = np.random.default_rng(seed)
    cache = {}
    out = []
    for i in range(n_ops):
        kind = ["cart", "spiral", "cs"][rng.choice(3, p=[0.4, 0.4, 0.2])]
        n = int(rng.choice(sizes))
        nc = int(rng.integers(coils[0], coils[1] + 1))
        if i == 0:
            kind, n, nc = "spiral", max(sizes), coils[1]
        elif i == 1:
            kind, n, nc = "cart", min(sizes), coils[0]
        r = np.random.default_rng(seed * 1000 + i)
        maps = workloads.coil_maps(n, n, nc, r)
        psi = workloads.noise_cov(nc, r)
        kw = dict(ny=n, nx=n, maps=torch.from_numpy(maps.astype(np.complex64)).to(dev), psi=psi,
                  probe_tile=0, graph=1)
        if kind == "cart":
            kw.update(mask=torch.from_numpy(workloads.cart_mask_1d(n, 2, 24)).to(dev), cg_iters=30)
        elif kind == "spiral":
            if ("traj", n) not in cache:
                cache[("traj", n)] = torch.from_numpy(workloads.spiral_traj(n, 2).astype(np.float32)).to(dev)
            traj = cache[("traj", n)]
            kw.update(mask=None, sampling=2, lam=0.1, cg_iters=30, traj=traj, nsamples=traj.shape[0])
        else:
            if ("pd", n) not in cache:
                cache[("pd", n)] = workloads.poisson_disc_mask(n, n, 2.0, 24, seed=n)
            mask = cache[("pd", n)]
            x = workloads.phantom(n, r)
            kd = cs_kspace_arrays(torch, dev, maps, psi, mask, x, 45.0, seed=i)
            kw.update(mask=torch.from_numpy(mask).to(dev), sampling=1, recon=1, kdata=kd,
                      fista_iters=100, cs_lambda=1e-3, wavelet_levels=4)
        out.append({"kind": kind, "n": n, "nc": nc, "kw": kw})
    return out


def serve_requests(np, pool, n_req, probes, seed=0):
    """Requests: an operator of the pool (uniform), a probe count from ``probes``."""
    rng = np.random.default_rng(seed + 7)
    out = []
    for i in range(n_req):
        j = int(rng.integers(len(pool)))
        out.append(dict(pool[j], op=j, probes=int(rng.choice(probes))))
    return out


def serve_run(lib, torch, dev, srv, reqs, arrivals=None, seed=0):
    """Submit the requests to the server (at the given arrival times in s, else
    one after the other, each waiting for the previous); returns (per-request
    info in submission order, accumulators)."""
    import threading
    accs = [[torch.zeros(r["n"] * r["n"], dtype=torch.float64, device=dev) for _ in range(2)]
            for r in reqs]
    torch.cuda.synchronize()
    ids = [None] * len(reqs)
    err = []

    def feeder():
        t0 = time.perf_counter()
        try:
            for i, r in enumerate(reqs):
                if arrivals is not None:
                    dt = arrivals[i] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                ids[i] = srv.submit(seed + i, 0, r["probes"], lib.make_accum(accs[i][0], None, accs[i][1]),
                                    **r["kw"])
                if arrivals is None:
                    srv.wait_idle(600.0)
        except Exception as e:     # reported by the caller
            err.append(e)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    if err:
        raise err[0]
    srv.wait_idle(600.0)
    done = {d["id"]: d for d in srv.poll(len(reqs) + 8)}
    torch.cuda.synchronize()
    return [done[i] for i in ids], accs


def _lat_stats(np, info):
    lat = np.array([d["t_done_ms"] - d["t_submit_ms"] for d in info])
    if lat.size == 0:
        return None
    return {"n": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2), "mean_ms": round(float(lat.mean()), 2)}


def serve_leg(lib, workloads, torch, np, dev, n_req=24, rhos=(0.5, 0.7, 0.9, 1.2), n_ops=10):
    """Serving mix over the stated ranges (matrix 128-384, coils 8-32, probes
    64-512; Cartesian / spiral / CS): a pool of distinct operators, tile shapes
    from the autotuner, graph replay, resident operators.  Cold pass (every
    operator built), warm sequential pass (capacity), then Poisson arrivals at
    rho x capacity on the same server: p50 / p99 latency, cold and warm."""
    import tempfile
    sizes, coils, probes = [128, 160, 192, 256, 288, 320, 384], (8, 32), [64, 128, 256, 512]
    budget, slots, depth = 96 << 30, 4, 2
    pool = serve_pool(workloads, torch, np, dev, n_ops, sizes, coils)
    tune_path = os.path.join(tempfile.mkdtemp(prefix="pico_tune_"), "tiles.txt")
    t0 = time.perf_counter()
    tuned = []
    for op in pool:
        d, keep = lib.make_desc(**dict(op["kw"], probe_tile=1))
        t = lib.pico_autotune(d, 16 << 30, tune_path)
        tuned.append({"kind": op["kind"], "n": op["n"], "coils": op["nc"], "probe_tile": t["probe_tile"],
                      "normal_form": t["normal_form"], "graph": t["graph"],
                      "probes_per_s": round(t["probes_per_s"], 1)})
    tune_s = time.perf_counter() - t0
    progress(f"serving: tuned {len(pool)} operators in {tune_s:.1f} s")
    reqs = serve_requests(np, pool, n_req, probes)
    srv = lib.Server(budget, slots, depth)
    srv.set_tuning(tune_path)
    cold_reqs = [dict(op, op=j, probes=64) for j, op in enumerate(pool)]
    cold, _ = serve_run(lib, torch, dev, srv, cold_reqs, seed=500)
    assert all(d["status"] == 0 for d in cold), [d["error"] for d in cold if d["status"]]
    seq, ref = serve_run(lib, torch, dev, srv, reqs)
    assert all(d["status"] == 0 for d in seq), [d["error"] for d in seq if d["status"]]
    service = [d["t_done_ms"] - d["t_admit_ms"] for d in seq]
    capacity = 1e3 / float(np.mean(service))
    rates = []
    progress(f"serving: warm capacity {capacity:.2f} requests/s")
    for rho in rhos:
        progress(f"serving: rho {rho}")
        lam = rho * capacity
        arr = np.cumsum(np.random.default_rng(int(rho * 1000)).exponential(1.0 / lam, n_req))
        info, accs = serve_run(lib, torch, dev, srv, reqs, arrivals=arr)
        assert all(d["status"] == 0 for d in info), [d["error"] for d in info if d["status"]]
        wait = np.array([d["t_admit_ms"] - d["t_submit_ms"] for d in info])
        span = (max(d["t_done_ms"] for d in info) - min(d["t_submit_ms"] for d in info)) / 1e3
        same = all(torch.equal(a, b) for x, y in zip(accs, ref) for a, b in zip(x, y))
        rates.append({"rho": rho, "arrival_rate_per_s": round(lam, 3), **_lat_stats(np, info),
                      "warm": _lat_stats(np, [d for d in info if d["op_reused"]]),
                      "cold": _lat_stats(np, [d for d in info if not d["op_reused"]]),
                      "mean_queue_wait_ms": round(float(wait.mean()), 2), "makespan_s": round(span, 3),
                      "probe_solves_per_s": round(sum(r["probes"] for r in reqs) / span, 1),
                      "results_identical_to_sequential": bool(same)})
    cache = srv.cache_stats()
    srv.close()
    kinds = {k: sum(r["kind"] == k for r in reqs) for k in ("cart", "spiral", "cs")}
    return {
        "workload": f"{n_req} requests per rate over a pool of {n_ops} operators (request kinds {kinds}), "
                    f"matrix {sizes}, coils U{{{coils[0]}..{coils[1]}}}, probes {probes}; Poisson arrivals at "
                    f"rho x the warm sequential capacity; budget {budget >> 30} GiB, {slots} slots, {depth} "
                    "tiles in flight; autotuned tiles, graph replay, resident operators",
        "pool": tuned, "autotune_s": round(tune_s, 2),
        "cold_first_requests": _lat_stats(np, cold),
        "capacity_req_per_s": round(capacity, 3),
        "mean_service_ms": round(float(np.mean(service)), 2),
        "rates": rates,
        "resident_cache": cache,
    }


def graph_leg(lib, workloads, torch, np, dev, steps=10):
    """ms per probe tile with graph replay against direct launches, on a
    launch-bound serving-sized operator (128^2, 8 coils) and on the headline one."""
    out = {}
    for name, cfg in (("cart1d_128x128x8_K64_cg30", dict(i=2, ny=128, nx=128, nc=8, K=64)),
                      ("cart1d_320x320x15_K256_cg30", dict(i=2, ny=320, nx=320, nc=15, K=256))):
        pr = workloads.config(cfg["i"], seed=0, ny=cfg["ny"], nx=cfg["nx"], nc=cfg["nc"])
        maps = torch.from_numpy(pr.maps.astype(np.complex64)).to(dev)
        mask = torch.from_numpy(pr.mask).to(dev)
        res = {}
        for g in (0, 1):
            h = lib.pico_init(pr.ny, pr.nx, maps, pr.psi, mask, cg_iters=30, probe_tile=cfg["K"], graph=g)
            at = [torch.zeros(pr.ny * pr.nx, dtype=torch.float64, device=dev) for _ in range(2)]
            acc = lib.make_accum(at[0], None, at[1])
            lib.pico_noise_map(h, 3, 0, cfg["K"], 0, acc)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                lib.pico_noise_map(h, 3, (i + 1) * cfg["K"], cfg["K"], 0, acc)
            e1.record()
            torch.cuda.synchronize()
            res["graph" if g else "direct"] = round(e0.elapsed_time(e1) / steps, 4)
            lib.pico_destroy(h)
        res["speedup"] = round(res["direct"] / res["graph"], 4)
        out[name] = {"ms_per_tile": res}
    return out


def plain_leg(torch, np, dev, prob, ref, max_probes=1024, check=None):
    """The plain FP32 per-probe form of the same estimator, for comparison
    with the batched / mixed-precision library path: one probe at a time,
    CG-SENSE with torch.fft (centred orthonormal 2-D FFT per coil, coils
    batched in one tensor), FP32 inner products and step scalars, an FP32
    accumulator, no fusion and no graph.  Probes are random phase from
    torch's generator (the same distribution as the library's).  Runs until
    the std map is within 1 % of the exact reference (checked every 32
    probes) or max_probes.  check = (lib, handle): the library's pico_apply_cov
    on the first 8 plain probes, for the maps' agreement."""
    ny, nx, nc = prob.ny, prob.nx, prob.nc
    L = np.linalg.cholesky(prob.psi)
    sw = np.linalg.solve(L, prob.maps.reshape(nc, -1)).reshape(nc, ny, nx)
    S = torch.from_numpy(sw.astype(np.complex64)).to(dev)
    P = torch.from_numpy(np.broadcast_to(prob.mask[:, None], (ny, nx)).astype(np.float32)).to(dev)

    def fc(x):
        return torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(x, dim=(-2, -1)), norm="ortho"), dim=(-2, -1))

    def fch(x):
        return torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(x, dim=(-2, -1)), norm="ortho"), dim=(-2, -1))

    def normal(p):
        return torch.sum(S.conj() * fch(P * fc(S * p)), dim=0)

    def solve(b):
        x = torch.zeros_like(b)
        r = b.clone()
        pp = r.clone()
        rr = torch.vdot(r.flatten(), r.flatten()).real
        for _ in range(prob.cg_iters):
            q = normal(pp)
            alpha = rr / torch.vdot(pp.flatten(), q.flatten()).real
            x = x + alpha * pp
            r = r - alpha * q
            rr_new = torch.vdot(r.flatten(), r.flatten()).real
            pp = r + (rr_new / rr) * pp
            rr = rr_new
        return x

    gen = torch.Generator(device=dev)
    gen.manual_seed(1234)
    acc = torch.zeros((ny, nx), dtype=torch.float32, device=dev)
    s_ref = torch.sqrt(torch.clamp(ref, min=0.0)).reshape(ny, nx)
    first = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, hit, e = 0, None, None
    while done < max_probes:
        v = torch.exp(2j * math.pi * torch.rand((ny, nx), generator=gen, device=dev)).to(torch.complex64)
        if check is not None and done < 8:
            first.append(v)
        acc += (v.conj() * solve(v)).real
        done += 1
        if done % 32 == 0:
            sd = torch.sqrt(torch.clamp(acc.double() / done, min=0.0))
            e = float(torch.linalg.norm(sd - s_ref) / torch.linalg.norm(s_ref))
            if e <= 0.01:
                hit = (time.perf_counter() - t0, done)
                break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = {"form": "plain FP32 per-probe (torch.fft, FP32 dots and accumulator, K=1, no graph)",
           "probe_solves_per_s": round(done / wall, 2), "probes": done,
           "time_to_1pct_s": round(hit[0], 4) if hit else None, "n_at_1pct": hit[1] if hit else None,
           "nrmse_at_stop": round(e, 5) if e is not None else None}
    if check is not None:
        lib, h = check
        vb = torch.stack(first)
        ub = torch.empty_like(vb)
        lib.pico_apply_cov(h, vb, ub, vb.shape[0])
        m_lib = (vb.conj() * ub).real.double().sum(0)
        m_plain = torch.zeros_like(m_lib)
        for v in first:
            m_plain += (v.conj() * solve(v)).real.double()
        torch.cuda.synchronize()
        res["map_rel_diff_vs_library_8_probes"] = float(torch.linalg.norm(m_plain - m_lib) / torch.linalg.norm(m_lib))
    return res


def stream_ceiling(torch, dev):
    """Practical HBM rates of plain torch streams over 2 GiB buffers (fill,
    copy, sum, axpy): the ceiling a streaming kernel can reach on this GPU,
    beside the published 8 TB/s."""
    n = 1 << 28
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.fill_(2.0)
    torch.cuda.synchronize()

    def rate(fn, nbytes, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9, 1)

    nb = n * 8
    out = {"write_GBs": rate(lambda: a.fill_(3.0), nb), "copy_GBs": rate(lambda: b.copy_(a), 2 * nb),
           "read_GBs": rate(lambda: a.sum(), nb), "axpy_GBs": rate(lambda: b.add_(a, alpha=0.5), 3 * nb)}
    del a, b
    torch.cuda.empty_cache()
    return out


def dense_leg(lib, torch, np, dev, prob, form=2, steps=3, ref=None):
    """The main workload with the dense per-column normal operator on the
    matrix cores: normal_form 2 (FP32 products) or 3 (FP16 products of split
    FP32 operands, three per product, FP32 accumulation).  Throughput, and the
    roofline of its CG-iteration kernel: the FP32 matrix peak for form 2 (8
    ny^2 flops per probe and column); for form 3, whose three FP16 products
    take a fraction of the time of the kernel's fused CG update, HBM: the
    update's 64 bytes per probe and pixel (x, r, p, q read and written) plus
    the blocks read once (8 ny^2 bytes per column), with the FP32-equivalent
    GEMM rate beside it."""
    ny, nx, K = prob.ny, prob.nx, 256
    maps = torch.from_numpy(prob.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    h = lib.pico_init(ny, nx, maps, prob.psi, mask, cg_iters=prob.cg_iters, probe_tile=K, normal_form=form)
    acc_keep = [torch.zeros(ny * nx, dtype=torch.float64, device=dev) for _ in range(2)]
    acc = lib.make_accum(*acc_keep)
    lib.pico_noise_map(h, 3, 0, K, 0, acc)
    torch.cuda.synchronize()
    lib.pico_profile_start(h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        lib.pico_noise_map(h, 3, K * (i + 1), K, 0, acc)
    e1.record()
    torch.cuda.synchronize()
    prof = lib.pico_profile_stop(h)
    ttt = None
    if ref is not None:   # time to 1 % NRMSE of the std map, as the main leg's (chunks of 32, monitor each)
        acc_t = [torch.zeros(ny * nx, dtype=torch.float64, device=dev) for _ in range(2)]
        acc2 = lib.make_accum(acc_t[0], None, acc_t[1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < 4096:
            lib.pico_noise_map(h, 7, done, 32, 0, acc2)
            done += 32
            if lib.pico_monitor_nrmse(h, acc2, ref) <= 0.01:
                ttt = {"time_to_1pct_s": round(time.perf_counter() - t0, 5), "n_at_1pct": done}
                break
    lib.pico_destroy(h)
    it_ms, it_n = prof["normal_iter"]
    avg_s = it_ms / it_n / 1e3
    flops = 8.0 * ny * ny * K * nx
    rate = steps * K / (e0.elapsed_time(e1) / 1e3)
    if form == 2:
        return {"form": "dense per-column blocks on the FP32 matrix cores (normal_form 2)",
                "probe_solves_per_s": round(rate, 2),
                "roofline": {"bound": "mfma", "achieved": round(flops / avg_s / 1e12, 2), "peak": PEAK_FP32_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(flops / avg_s / 1e12 / PEAK_FP32_TFLOPS, 4),
                             "kernel": "k_cart1d_gram<C1_ITER>", "avg_launch_us": round(avg_s * 1e6, 2),
                             "flops_per_launch": flops}}
    nbytes = 64.0 * ny * nx * K + 8.0 * ny * ny * nx
    traffic = None   # counter-measured HBM bytes, while the kernel sources match the measured ones
    tfile = os.path.join(ROOT, "profiles", "traffic_gram16_iter_cart1d_320x320x15_K256.json")
    if (ny, nx, K) == (320, 320, 256) and os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("kernel_src_sha") == gram16_source_digest():
            traffic = tj.get("hbm_bytes_per_launch")
    return {"form": "dense per-column blocks, split-FP16 products on the FP16 matrix cores (normal_form 3)",
            "probe_solves_per_s": round(rate, 2), "time_to_1pct": ttt,
            "roofline": {"bound": "hbm", "achieved": round(nbytes / avg_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(nbytes / avg_s / 1e9 / PEAK_HBM_GBS, 4), "traffic": traffic,
                         "kernel": "k_cart1d_gram16<C1_ITER>", "avg_launch_us": round(avg_s * 1e6, 2),
                         "bytes_per_launch": nbytes,
                         "gemm_tflops_fp32_equivalent": round(flops / avg_s / 1e12, 2)}}


def reduced_leg(lib, torch, np, dev, prob, ref, factor=2, max_probes=1024):
    """Reduced-resolution grid (Sec. 5, Discussion) on the main workload: the
    coarse operator of the same acquisition, its map upsampled to the native
    grid and compared with the native exact map.  Reports the floor (the
    exact coarse map, upsampled), the coarse throughput, and the NRMSE curve
    of the probed map (chunks of 32 probes; finalize + upsample + NRMSE inside
    the timed loop)."""
    ny, nx = prob.ny, prob.nx
    cy, cx = ny // factor, nx // factor
    maps = torch.from_numpy(prob.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    h = lib.pico_init_reduced(factor, ny, nx, maps, prob.psi, mask, cg_iters=prob.cg_iters, probe_tile=256)
    s_ref = torch.sqrt(torch.clamp(ref, min=0.0))

    def nrmse(var_native):
        return float(torch.linalg.norm(torch.sqrt(torch.clamp(var_native, min=0.0)) - s_ref) / torch.linalg.norm(s_ref))

    vc = torch.empty(cy * cx, dtype=torch.float64, device=dev)
    up = torch.empty(ny * nx, dtype=torch.float64, device=dev)
    lib.pico_exact_diag(h, vc)
    lib.pico_upsample_map(h, vc, up)
    floor = nrmse(up)
    acc_t = [torch.zeros(cy * cx, dtype=torch.float64, device=dev) for _ in range(2)]
    acc = lib.make_accum(acc_t[0], None, acc_t[1])
    warm_t = [torch.zeros(cy * cx, dtype=torch.float64, device=dev) for _ in range(2)]
    lib.pico_noise_map(h, 17, 0, 256, 0, lib.make_accum(*warm_t))   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve, done = [], 0
    while done < max_probes:
        lib.pico_noise_map(h, 17, done, 32, 0, acc)
        done += 32
        lib.pico_finalize(h, acc, vc)
        lib.pico_upsample_map(h, vc, up)
        curve.append((done, round(time.perf_counter() - t0, 5), round(nrmse(up), 5)))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lib.pico_noise_map(h, 17, done, 256, 0, acc)
    e1.record()
    torch.cuda.synchronize()
    lib.pico_destroy(h)
    hit3 = next(((n, t) for n, t, e in curve if e <= 0.03), None)
    return {"workload": f"factor {factor}: coarse {cy}x{cx} of the native {ny}x{nx} acquisition "
                        "(central k-space block), periodic bilinear upsampling",
            "floor_nrmse_exact_coarse": round(floor, 5),
            "coarse_probe_solves_per_s": round(256 / (e0.elapsed_time(e1) / 1e3), 2),
            "time_to_3pct_s": hit3[1] if hit3 else None, "n_at_3pct": hit3[0] if hit3 else None,
            "nrmse_curve": [c for c in curve if c[0] in (32, 64, 128, 192, 256, 512, 1024)]}


def spiral_leg(lib, workloads, torch, np, dev, steps, storage):
    """Probe-solves/s of the spiral workload and the HBM roofline of its
    Toeplitz normal operator; storage PICO_BF16_STREAM keeps maps and the
    row-transformed coil planes in bfloat16 (half the plane bytes)."""
    sp = workloads.config(3, seed=0)
    Ks = 256
    traj = torch.from_numpy(sp.traj.astype(np.float32)).to(dev)
    smaps = torch.from_numpy(sp.maps.astype(np.complex64)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = lib.pico_init(sp.ny, sp.nx, smaps, sp.psi, None, sampling=lib.PICO_NONCART,
                       lam=sp.lam, cg_iters=sp.cg_iters, probe_tile=Ks, traj=traj,
                       nsamples=traj.shape[0], storage=storage)
    sinit = time.perf_counter() - t0
    ns = sp.ny * sp.nx
    sacc_t = [torch.zeros(ns, dtype=torch.float64, device=dev) for _ in range(2)]
    sacc = lib.make_accum(*sacc_t)
    lib.pico_noise_map(hs, 5, 0, Ks, 0, sacc)            # warm-up step
    torch.cuda.synchronize()
    lib.pico_profile_start(hs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        lib.pico_noise_map(hs, 5, (i + 1) * Ks, Ks, 0, sacc)
    e1.record()
    torch.cuda.synchronize()
    sprof = lib.pico_profile_stop(hs)
    lib.pico_destroy(hs)
    sms = e0.elapsed_time(e1) / steps
    it_ms, it_n = sprof["normal_iter"]
    sop_s = it_ms / it_n / 1e3
    Gx = 2 * sp.nx
    # per probe and normal-operator application: T written, read+written, read
    # (nc ny Gx elements of 8 B, or 4 B in bfloat16) + per-probe fields (rows
    # pass: x r p q in, x r p out; inverse pass: p r in, q out) + maps twice
    # per launch
    eb = 4 if storage == lib.PICO_BF16_STREAM else 8
    t_bytes = 4 * sp.nc * sp.ny * Gx * eb
    f_bytes = 10 * ns * 8
    sbytes = Ks * (t_bytes + f_bytes) + 2 * sp.nc * ns * (4 if storage else 8)
    return {
        "workload": "spiral 256x256, 16 coils, 48x4096 interleaves R=2 (98304 samples), "
                    "lambda 0.1, K=256 probes, CG 30 per solve (2 solves + 1 M per probe)",
        "storage": ["f32", "bf16 maps", "bf16 maps + planes"][storage],
        "probe_solves_per_s": round(Ks / (sms / 1e3), 2), "ms_per_step": round(sms, 3),
        "init_s": round(sinit, 3),
        "roofline": {"bound": "hbm", "achieved": round(sbytes / sop_s / 1e9, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(sbytes / sop_s / 1e9 / PEAK_HBM_GBS, 4),
                     "kernel": "grid normal operator (rows_fwd + cols + rows_inv), C1_ITER",
                     "avg_application_us": round(sop_s * 1e6, 1), "alg_bytes": sbytes},
        "kernel_ms": {k: round(v[0], 3) for k, v in sprof.items()},
    }


def spiral_subset_exact(lib, torch, h, n_side, voxels, K=256):
    """Exact Sigma_jj (and the off-diagonal energies of column j) for the
    voxels j of ``voxels`` (a multiple of K of them): unit-vector right-hand
    sides e_j through pico_apply_cov, K per launch (Sigma e_j is column j of
    Sigma).  Returns (diag, sum_{l != j} |Sigma_lj|^2, sum_{l != j} (Re Sigma_lj)^2)
    as float64 tensors on the device."""
    n = n_side * n_side
    dev = voxels.device
    ar = torch.arange(K, device=dev)
    diag, off, off_re = [], [], []
    v = torch.zeros((K, n), dtype=torch.complex64, device=dev)
    u = torch.empty_like(v)
    for c0 in range(0, voxels.numel(), K):
        idx = voxels[c0:c0 + K]
        v.zero_()
        v[ar, idx] = 1.0
        lib.pico_apply_cov(h, v, u, K)
        ud = u[ar, idx]
        uu = u.to(torch.complex128)
        d = ud.real.to(torch.float64)
        diag.append(d)
        off.append((uu.abs() ** 2).sum(dim=1) - ud.to(torch.complex128).abs() ** 2)
        off_re.append((uu.real ** 2).sum(dim=1) - d ** 2)
    return torch.cat(diag), torch.cat(off), torch.cat(off_re)


def spiral_exact_leg(lib, workloads, torch, np, dev, Rs=(2, 3, 4), n_vox=4096, chunk=128, max_n=32768,
                     families=True):
    """Time to a 1 % std map on the spiral workload at R = 2, 3, 4 (the
    paper's non-Cartesian comparison, Sec. 3.2.2) against an exact
    reference: Sigma_jj by unit-vector solves on a seeded random subset of
    n_vox voxels, so the NRMSE of the std maps is taken over that subset (an
    unbiased sample of the full-FOV sums).  PICO (seed 7) and PMR (noise
    replicas through the gridding adjoint, seed 3) add samples in chunks;
    the clocks include the monitor.  At R = 2 also the probe families
    (Sec. 2.2, Eqs. (18)-(20)): probes to 1 %, and the per-voxel variance of
    the probe terms Re(conj v_j (Sigma v)_j) against the closed forms of
    App. B (random phase and QPSK: 1/2 sum_{l != j} |Sigma_jl|^2; complex
    Gaussian: Sigma_jj^2 + 1/2 sum_{l != j} |Sigma_jl|^2; real Rademacher:
    sum_{l != j} (Re Sigma_jl)^2)."""
    out = {}
    for R in Rs:
        progress(f"spiral R = {R}")
        sp = workloads.config(3, seed=0, R=R)
        traj = torch.from_numpy(sp.traj.astype(np.float32)).to(dev)
        smaps = torch.from_numpy(sp.maps.astype(np.complex64)).to(dev)
        h = lib.pico_init(sp.ny, sp.nx, smaps, sp.psi, None, sampling=lib.PICO_NONCART, lam=sp.lam,
                          cg_iters=sp.cg_iters, probe_tile=256, traj=traj, nsamples=traj.shape[0],
                          oversamp=2.0, kb_width=6)
        n = sp.ny * sp.nx
        vox = torch.from_numpy(np.sort(np.random.default_rng(1000 + R).choice(n, n_vox, replace=False))).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref, off, off_re = spiral_subset_exact(lib, torch, h, sp.ny, vox)
        torch.cuda.synchronize()
        ref_s = time.perf_counter() - t0
        s_ref = torch.sqrt(torch.clamp(ref, min=0.0))

        def nrmse(var_sub):
            return float(torch.linalg.norm(torch.sqrt(torch.clamp(var_sub, min=0.0)) - s_ref) /
                         torch.linalg.norm(s_ref))

        def run(kind, seed, dist=0):
            at = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
            acc = lib.make_accum(*at)
            var = torch.empty(n, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done, hit, e = 0, None, None
            while done < max_n:
                if kind == "pico":
                    lib.pico_noise_map(h, seed, done, chunk, dist, acc)
                    done += chunk
                    e = nrmse(at[0][vox] / done)
                else:
                    lib.pico_pmr_baseline(h, seed, done, chunk, acc)
                    done += chunk
                    lib.pico_pmr_finalize(h, acc, var)
                    e = nrmse(var[vox])
                if e <= 0.01:
                    hit = (time.perf_counter() - t0, done)
                    break
            return hit, e, at, done

        (ph, pe, pat, pn) = run("pico", 7)
        (mh, me, _, _) = run("pmr", 3)
        res = {"samples": int(traj.shape[0]), "reference": f"exact Sigma_jj on {n_vox} seeded voxels "
                                                        f"({n_vox // 256} launches of 256 unit vectors, {ref_s:.2f} s)",
               "pico_time_to_1pct_s": round(ph[0], 4) if ph else None, "pico_n_at_1pct": ph[1] if ph else None,
               "pico_nrmse_at_stop": round(pe, 5),
               "pmr_time_to_1pct_s": round(mh[0], 4) if mh else None, "pmr_n_at_1pct": mh[1] if mh else None,
               "pmr_nrmse_at_stop": round(me, 5),
               "speedup_pico_vs_pmr": round(mh[0] / ph[0], 3) if (ph and mh) else None}
        if families and R == Rs[0]:
            pred = {"random_phase": 0.5 * off, "qpsk": 0.5 * off, "gaussian": ref ** 2 + 0.5 * off,
                    "rademacher": off_re}
            fam = {}
            for name, dist in (("random_phase", 0), ("qpsk", 1), ("rademacher", 2), ("gaussian", 3)):
                hit, e, at, N = run("pico", 41, dist)
                m = at[0][vox] / N
                s2 = (at[2][vox] - N * m * m) / (N - 1)
                ratio = float((s2 / pred[name]).mean())
                fam[name] = {"n_at_1pct": hit[1] if hit else None, "nrmse_at_stop": round(e, 5),
                             "probe_term_var_over_closed_form": round(ratio, 4), "probes_for_ratio": N}
            res["probe_families"] = fam
        lib.pico_destroy(h)
        out[f"R{R}"] = res
    out["workload"] = ("spiral 256x256, 16 coils, 48x4096 interleaves subsampled by R, lambda 0.1, CG 30 per solve, "
                       "K=256; Kaiser-Bessel gridding (2.0, W 6) for the PMR data path; samples in chunks of "
                       f"{chunk}")
    out["paper_context"] = ("paper, GE spiral phantom on its own hardware: 64.0 / 70.6 / 91.0 s (PICO) vs "
                            "462.6 / 501.0 / 538.6 s (PMR) at R = 2 / 3 / 4")
    return out


def spiral_gridding_leg(lib, workloads, torch, np, dev, steps=1):
    """The spiral workload (R=2, K=256) with the gridding normal operator
    (Kaiser-Bessel sigma 2, W 6, binned tile interpolation/spread) instead of
    the Toeplitz one: probe-solves/s, per-application time, and its HBM
    roofline on the algorithmic bytes (per coil and probe, G^2 complex64
    points: the image rows' row transforms written (half the grid), read by the
    column transforms, which write the full grid; the stencil reads and writes
    it; the inverse column transforms read it and write the image rows, which
    the inverse row transforms read: 6 half-or-full grids, 48 G^2 bytes; the
    image row read and the combined q read and written, 24 B per pixel; plus
    the probe fields), and ||Sigma_grid v - Sigma_T v|| / ||Sigma_T v|| over
    one tile of K random-phase probes (every launch of the leg is a K-probe
    one)."""
    sp = workloads.config(3, seed=0)
    traj = torch.from_numpy(sp.traj.astype(np.float32)).to(dev)
    smaps = torch.from_numpy(sp.maps.astype(np.complex64)).to(dev)
    K = 256
    n = sp.ny * sp.nx
    kw = dict(sampling=lib.PICO_NONCART, lam=sp.lam, cg_iters=sp.cg_iters, probe_tile=K, traj=traj,
              nsamples=traj.shape[0], oversamp=2.0, kb_width=6)
    h = lib.pico_init(sp.ny, sp.nx, smaps, sp.psi, None, noncart_normal=1, **kw)
    at = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
    acc = lib.make_accum(at[0], None, at[1])
    lib.pico_noise_map(h, 3, 0, K, 0, acc)
    torch.cuda.synchronize()
    lib.pico_profile_start(h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        lib.pico_noise_map(h, 3, (i + 1) * K, K, 0, acc)
    e1.record()
    torch.cuda.synchronize()
    prof = lib.pico_profile_stop(h)
    ms = e0.elapsed_time(e1) / steps
    v = torch.from_numpy(np.exp(2j * np.pi * np.random.default_rng(4).random((K, n))).astype(np.complex64)).to(dev)
    ug = torch.empty_like(v)
    lib.pico_apply_cov(h, v, ug, K)
    lib.pico_destroy(h)
    ht = lib.pico_init(sp.ny, sp.nx, smaps, sp.psi, None, noncart_normal=0, **kw)
    ut = torch.empty_like(v)
    lib.pico_apply_cov(ht, v, ut, K)
    torch.cuda.synchronize()
    lib.pico_destroy(ht)
    rel = float(torch.linalg.norm(ug - ut) / torch.linalg.norm(ut))
    it_ms, it_n = prof["normal_iter"]
    op_s = it_ms / it_n / 1e3
    G = 2 * sp.ny
    alg = K * sp.nc * (48 * G * G + 24 * n) + K * 4 * 8 * n
    return {"workload": "spiral 256x256, 16 coils, 48x4096 R=2, lambda 0.1, CG 30, K=256; gridding normal "
                        "operator (sigma 2, W 6, 16x16 tile bins)",
            "probe_solves_per_s": round(K / (ms / 1e3), 2), "ms_per_step": round(ms, 3),
            "sigma_rel_diff_vs_toeplitz_256_probes": rel,
            "roofline": {"bound": "hbm", "achieved": round(alg / op_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(alg / op_s / 1e9 / PEAK_HBM_GBS, 4),
                         "kernel": "gridding normal operator (expand + row FFTs, column FFTs, stencil, "
                                   "inverse column FFTs, inverse row FFTs + crop/combine), C1_ITER",
                         "avg_application_us": round(op_s * 1e6, 1), "alg_bytes": alg},
            "kernel_ms": {k: round(v2[0], 3) for k, v2 in prof.items()}}


def true_residual(lib, torch, np, dev, h, prob, nprobe=4):
    """||v - M x|| / ||v|| for x = pico_apply_cov(v) (lambda = 0: x = CG_30(M, v))
    on nprobe random-phase probes, with M applied here in complex128 by torch:
    whitened maps L^-1 S (Cholesky of psi), centred orthonormal 2-D DFT, the
    phase-encode mask, its adjoint, coil combine.  The CG's own figure
    (cg_max_relres) comes from its residual recurrence."""
    ny, nx = prob.ny, prob.nx
    rng = np.random.default_rng(77)
    v = torch.from_numpy(np.exp(2j * np.pi * rng.random((nprobe, ny, nx))).astype(np.complex64)).to(dev)
    x = torch.empty_like(v)
    lib.pico_apply_cov(h, v, x, nprobe)
    torch.cuda.synchronize()
    Lc = torch.linalg.cholesky(torch.from_numpy(np.asarray(prob.psi, np.complex128)).to(dev))
    S = torch.from_numpy(np.asarray(prob.maps, np.complex128)).to(dev).reshape(prob.nc, -1)
    Sw = torch.linalg.solve_triangular(Lc, S, upper=False).reshape(prob.nc, ny, nx)
    P = torch.from_numpy(np.asarray(prob.mask, np.float64)).to(dev)[:, None]
    out = []
    for k in range(nprobe):
        xk = x[k].to(torch.complex128)
        cz = Sw * xk
        kz = torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(cz, dim=(-2, -1)), norm="ortho"), dim=(-2, -1))
        bz = torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(P * kz, dim=(-2, -1)), norm="ortho"),
                                dim=(-2, -1))
        mx = (torch.conj(Sw) * bz).sum(dim=0)
        vk = v[k].to(torch.complex128)
        out.append(float(torch.linalg.norm(vk - mx) / torch.linalg.norm(vk)))
    return {"max": max(out), "probes": nprobe,
            "note": "||v - M x|| / ||v|| with M applied in complex128 outside the library"}


def std_map_nrmse(torch, a, ref):
    """||sqrt(a) - sqrt(ref)|| / ||sqrt(ref)|| of two variance maps (std maps)."""
    sa, sr = torch.sqrt(torch.clamp(a, min=0.0)), torch.sqrt(torch.clamp(ref, min=0.0))
    return float(torch.linalg.norm(sa - sr) / torch.linalg.norm(sr))


def cs_leg(lib, workloads, torch, np, dev, steps, storage=0):
    """JVPs/s of the CS workload and the HBM roofline of its normal operator."""
    pr = workloads.config(4, seed=0)
    K = pr.probes
    n = pr.ny * pr.nx
    kd = cs_kspace(torch, dev, pr)
    maps = torch.from_numpy(pr.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(pr.mask).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = lib.pico_init(pr.ny, pr.nx, maps, pr.psi, mask, sampling=lib.PICO_CART_2D,
                      recon=lib.PICO_CS_FISTA_L1WAV, kdata=kd, fista_iters=pr.extra["fista_iters"],
                      cs_lambda=pr.extra["cs_lambda"], wavelet_levels=pr.extra["levels"], probe_tile=K,
                      storage=storage)
    init_s = time.perf_counter() - t0
    acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
    acc = lib.make_accum(*acc_t)
    lib.pico_noise_map(h, 3, 0, K, 0, acc)                   # warm-up step
    torch.cuda.synchronize()
    lib.pico_profile_start(h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        lib.pico_noise_map(h, 3, (i + 1) * K, K, 0, acc)
    e1.record()
    torch.cuda.synchronize()
    prof = lib.pico_profile_stop(h)
    lib.pico_destroy(h)
    vmap = acc_t[0].cpu()
    ms = e0.elapsed_time(e1) / steps
    it_ms, it_n = prof["normal_iter"]
    op_s = it_ms / it_n / 1e3
    # per probe and normal-operator application: coil k-space written, read+written,
    # read (nc ny nx elements of 8 B, 4 B in bfloat16) + p read, q written; maps
    # twice per launch
    eb = 4 if storage == lib.PICO_BF16_STREAM else 8
    alg = K * (4 * pr.nc * n * eb + 2 * n * 8) + 2 * pr.nc * n * (4 if storage else 8)
    return {
        "workload": f"CS {pr.ny}x{pr.nx}, {pr.nc} coils, Poisson-disc R=2 (24x24 calib), "
                    f"L1-db4 (4 levels) FISTA {pr.extra['fista_iters']} its, lambda "
                    f"{pr.extra['cs_lambda']}, K={K} JVP probes per step",
        "storage": ["f32", "bf16 maps", "bf16 maps + planes"][storage],
        "jvps_per_s": round(K / (ms / 1e3), 2), "ms_per_step": round(ms, 3),
        "init_s": round(init_s, 3),
        "roofline": {"bound": "hbm", "achieved": round(alg / op_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(alg / op_s / 1e9 / PEAK_HBM_GBS, 4),
                     "kernel": "grid normal operator (rows_fwd + cols + rows_inv), C1_APPLY",
                     "avg_application_us": round(op_s * 1e6, 1), "alg_bytes": alg},
        "kernel_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "_map": vmap, "probes_accumulated": K * (steps + 1),
    }


def cs_tv_leg(lib, workloads, torch, np, dev, steps, n_conv=5000, storage=0, pmr=True):
    """The paper's CS model (Sec. 3.2.3): TV-regularised FISTA, 320 x 320, 15
    coils, Poisson-disc R=2, lambda_TV 1e-2, 100 iterations (10 dual steps per
    prox).  Jacobian probes per second (K per step) against FP64 PMR replicas
    per second on the same operator, and the time each needs for the paper's
    converged sample count (5000 for both methods, its appendix on references)."""
    pr = workloads.config(4, seed=0, reg="tv")
    K = pr.probes
    n = pr.ny * pr.nx
    kd = cs_kspace(torch, dev, pr)
    maps = torch.from_numpy(pr.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(pr.mask).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = lib.pico_init(pr.ny, pr.nx, maps, pr.psi, mask, sampling=lib.PICO_CART_2D,
                      recon=lib.PICO_CS_FISTA_TV, kdata=kd, fista_iters=pr.extra["fista_iters"],
                      cs_lambda=pr.extra["cs_lambda"], tv_inner_iters=pr.extra["tv_inner"], probe_tile=K,
                      storage=storage)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    resident, _ = lib.pico_op_bytes(h)
    acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
    acc = lib.make_accum(*acc_t)
    lib.pico_noise_map(h, 3, 0, K, 0, acc)                   # warm-up step
    torch.cuda.synchronize()
    lib.pico_profile_start(h)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        lib.pico_noise_map(h, 3, (i + 1) * K, K, 0, acc)
    e1.record()
    torch.cuda.synchronize()
    prof = lib.pico_profile_stop(h)
    ms = e0.elapsed_time(e1) / steps
    # PMR: one batch of FP64 replicas (the finite difference at a small sigma needs FP64)
    nrep = 16
    pmr_s = None
    if pmr:
        pacc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        pacc = lib.make_accum(*pacc_t)
        lib.pico_pmr_cs(h, 5, 0, 4, 1e-3, pacc)                  # workspace + warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.pico_pmr_cs(h, 5, 4, nrep, 1e-3, pacc)
        torch.cuda.synchronize()
        pmr_s = (time.perf_counter() - t0) / nrep
    lib.pico_destroy(h)
    vmap = acc_t[0].cpu()
    jvps = K / (ms / 1e3)
    it_ms, it_n = prof["normal_iter"]
    op_s = it_ms / it_n / 1e3
    eb = 4 if storage == lib.PICO_BF16_STREAM else 8
    alg = K * (4 * pr.nc * n * eb + 2 * n * 8) + 2 * pr.nc * n * (4 if storage else 8)   # as the CS leg's
    # the TV tangent (the rest of the step): per prox, the library runs one
    # single step first when the count is odd, then passes of four dual steps
    # while four remain, then pairs.  The first pass starts from zero, reads dz
    # and writes dr, dp (40 B per tangent and pixel); each later pass reads dz,
    # dr, dp and writes dr, dp (72 B); the last pass of several steps writes
    # no dual field and ends with the FISTA step: x read and written, y
    # written (40 + 24 B; 8 + 24 B if it is also the first).  The gradient
    # point z = y - (q - g) / s^2 before the prox: 3 fields read, 1 written
    # (32 B).  The projection data (20 B per pixel and step) is shared by the
    # tangents of a workgroup and not counted.
    inner, T = pr.extra["tv_inner"], pr.extra["fista_iters"]
    passes, it = [], 0
    if inner % 2:
        passes.append(1)
        it = 1
    while inner - it >= 4 and pr.ny >= 25 and pr.nx >= 41:
        passes.append(4)
        it += 4
    while it < inner:
        passes.append(2)
        it += 2
    pass_bytes = [40 if j == 0 else 72 for j in range(len(passes))]
    if passes[-1] > 1:
        pass_bytes[-1] += 24 - 32
    else:
        pass_bytes.append(48)                     # a single step alone: separate FISTA step
    tv_bytes = T * K * n * (sum(pass_bytes) + 32)
    tv_s = prof["other"][0] / 1e3 / steps
    return {
        "workload": f"TV-CS {pr.ny}x{pr.nx}, {pr.nc} coils, Poisson-disc R=2 (24x24 calib), "
                    f"FISTA {pr.extra['fista_iters']} its x {pr.extra['tv_inner']} dual steps, lambda_TV "
                    f"{pr.extra['cs_lambda']}, K={K} JVP probes per step",
        "jvps_per_s": round(jvps, 2), "ms_per_step": round(ms, 3), "init_s": round(init_s, 3),
        "storage": ["f32", "bf16 maps", "bf16 maps + planes"][storage],
        "resident_bytes": int(resident),
        "pmr_replicas_per_s": round(1.0 / pmr_s, 2) if pmr_s else None, "pmr_precision": "f64",
        "n_converged": n_conv,
        "pico_s_at_n": round(n_conv / jvps, 2), "pmr_s_at_n": round(n_conv * pmr_s, 2) if pmr_s else None,
        "roofline": {"bound": "hbm", "achieved": round(alg / op_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(alg / op_s / 1e9 / PEAK_HBM_GBS, 4),
                     "kernel": "grid normal operator (rows_fwd + cols + rows_inv), C1_APPLY",
                     "avg_application_us": round(op_s * 1e6, 1), "alg_bytes": alg},
        "tv_tangent": {"bound": "hbm", "ms_per_step": round(tv_s * 1e3, 3), "passes_per_prox": passes,
                       "alg_bytes_per_step": tv_bytes,
                       "achieved_GBs": round(tv_bytes / tv_s / 1e9, 1),
                       "frac": round(tv_bytes / tv_s / 1e9 / PEAK_HBM_GBS, 4),
                       "note": "time of the step outside the normal-operator applications: the dual-step "
                               "kernels plus the FISTA momentum and gradient kernels"},
        "kernel_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "_map": vmap, "probes_accumulated": K * (steps + 1),
    }


def cs_converged_leg(lib, workloads, torch, np, dev, reg="l1wav", n_max=8192):
    """Time to converged accuracy of the Jacobian probes on a CS workload,
    measured with the reference protocol of the paper's appendix on reference
    budgets: a gold map of n_max probes (seed 201, maps and the clock kept at
    every power of two N >= K along the way); the estimate is converged at
    the smallest N whose doubling improves the std-map NRMSE against the gold
    by < 0.5 % and changes the FOV-mean variance by < 0.2 %, and the time to
    converged accuracy is the measured wall time to that N.  An independent
    run (seed 7) is also taken to the same NRMSE against the gold (it needs
    more probes: the nested maps share samples with the gold).  PMR (FP64
    replicas) is reported as its measured rate and the derived time for the
    same N."""
    tv = reg == "tv"
    pr = workloads.config(4, seed=0, reg="tv") if tv else workloads.config(4, seed=0)
    K = pr.probes
    n = pr.ny * pr.nx
    kd = cs_kspace(torch, dev, pr)
    maps = torch.from_numpy(pr.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(pr.mask).to(dev)
    kw = dict(sampling=lib.PICO_CART_2D, kdata=kd, fista_iters=pr.extra["fista_iters"],
              cs_lambda=pr.extra["cs_lambda"], probe_tile=K)
    if tv:
        kw.update(recon=lib.PICO_CS_FISTA_TV, tv_inner_iters=pr.extra["tv_inner"])
    else:
        kw.update(recon=lib.PICO_CS_FISTA_L1WAV, wavelet_levels=pr.extra["levels"])
    h = lib.pico_init(pr.ny, pr.nx, maps, pr.psi, mask, **kw)
    ga = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
    gacc = lib.make_accum(*ga)
    snaps, t_at = {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < n_max:
        lib.pico_noise_map(h, 201, done, K, 0, gacc)
        done += K
        if done & (done - 1) == 0:
            snaps[done] = ga[0] / done
            torch.cuda.synchronize()
            t_at[done] = time.perf_counter() - t0
    gold_s = t_at[n_max]
    gold = snaps[n_max]
    curve, n_conv, e_conv = [], None, None
    for N in sorted(snaps):
        if N == n_max:
            break
        e1, e2 = std_map_nrmse(torch, snaps[N], gold), std_map_nrmse(torch, snaps[2 * N], gold)
        r1, r2 = float(snaps[N].mean()), float(snaps[2 * N].mean())
        curve.append((N, round(e1, 5)))
        if n_conv is None and e1 - e2 < 0.005 and abs(r2 - r1) / abs(r2) < 0.002:
            n_conv, e_conv = N, e1
    res = {"workload": f"{'TV' if tv else 'L1-db4'} CS {pr.ny}x{pr.nx}, {pr.nc} coils, Poisson-disc R=2, "
                       f"FISTA {pr.extra['fista_iters']}, K={K} per tile",
           "gold": f"{n_max} probes ({gold_s:.2f} s)", "nrmse_vs_gold_by_n": curve,
           "n_converged": n_conv, "converged_nrmse": round(e_conv, 5) if e_conv is not None else None,
           "pico_time_to_converged_s": round(t_at[n_conv], 4) if n_conv else None}
    if n_conv is not None:
        at = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
        acc = lib.make_accum(*at)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, hit, e = 0, None, None
        while done < n_max:
            lib.pico_noise_map(h, 7, done, K, 0, acc)
            done += K
            e = std_map_nrmse(torch, at[0] / done, gold)
            if e <= e_conv:
                hit = (time.perf_counter() - t0, done)
                break
        res["independent_run_to_converged_nrmse"] = {"seconds": round(hit[0], 4) if hit else None,
                                                     "n": hit[1] if hit else None, "nrmse_at_stop": round(e, 5)}
        pa = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        pacc = lib.make_accum(*pa)
        lib.pico_pmr_cs(h, 5, 0, 4, 1e-3, pacc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.pico_pmr_cs(h, 5, 4, 16, 1e-3, pacc)
        torch.cuda.synchronize()
        rate = 16 / (time.perf_counter() - t0)
        res.update({"pmr_replicas_per_s": round(rate, 2),
                    "pmr_s_at_same_n_derived": round(n_conv / rate, 2)})
    lib.pico_destroy(h)
    res["paper_context"] = "paper, fastMRI knee TV-CS on its own hardware: 52.3 s (PICO) vs 95.5 s (PMR) at N = 5000"
    return res


def cs_robustness(lib, workloads, torch, np, dev, N=128, reg="l1wav"):
    """Noise-level sweep of the CS workload (Sec. 3.2.3, robustness): data at
    input SNR 45 dB - 20 log10(scale); per level the Jacobian-probe std map
    (N probes) against the PMR std map (N replicas perturbed at the data's own
    noise level, normalised by it); both per unit whitened noise.  reg "tv"
    sweeps the TV model of the paper's experiment."""
    pr = workloads.config(4, seed=0, reg=reg)
    tv = reg == "tv"
    n = pr.ny * pr.nx
    maps = torch.from_numpy(pr.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(pr.mask).to(dev)
    rows = []
    for scale in (1, 5, 10, 50, 100, 200):
        snr = 45.0 - 20.0 * math.log10(scale)
        kd = cs_kspace_arrays(torch, dev, pr.maps, pr.psi, pr.mask, pr.extra["phantom"], snr, seed=0)
        # whitened noise std of the data: the signal rms on the mask times 10^(-snr/20)
        xs = torch.from_numpy(pr.extra["phantom"].astype(np.complex128)).to(dev)
        mk = torch.from_numpy(pr.mask.astype(np.float64)).to(dev)
        k0 = torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(
            torch.from_numpy(pr.maps.astype(np.complex128)).to(dev) * xs[None], dim=(-2, -1)), norm="ortho"),
            dim=(-2, -1)) * mk[None]
        sigma = float(torch.sqrt(torch.mean(torch.abs(k0[:, mk > 0]) ** 2))) * 10 ** (-snr / 20)
        h = lib.pico_init(pr.ny, pr.nx, maps, pr.psi, mask, sampling=lib.PICO_CART_2D,
                          recon=lib.PICO_CS_FISTA_TV if tv else lib.PICO_CS_FISTA_L1WAV, kdata=kd,
                          fista_iters=pr.extra["fista_iters"], cs_lambda=pr.extra["cs_lambda"],
                          wavelet_levels=pr.extra["levels"], tv_inner_iters=pr.extra["tv_inner"],
                          probe_tile=128)
        a1 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        acc1 = lib.make_accum(*a1)
        t0 = time.perf_counter()
        lib.pico_noise_map(h, 3, 0, N, 0, acc1)
        e_pico = lib.pico_monitor_stderr(h, acc1)    # delta-method std-map error of the probe mean
        t_pico = time.perf_counter() - t0
        a2 = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        acc2 = lib.make_accum(*a2)
        t0 = time.perf_counter()
        for r0 in range(0, N, 256):
            lib.pico_pmr_cs(h, 5, r0, min(256, N - r0), sigma, acc2)
            torch.cuda.synchronize()
            progress(f"robustness {reg} {snr:.1f} dB: {min(N, r0 + 256)} / {N} replicas")
        t_pmr = time.perf_counter() - t0
        var = torch.empty(n, dtype=torch.float64, device=dev)
        lib.pico_pmr_finalize(h, acc2, var)
        torch.cuda.synchronize()
        lib.pico_destroy(h)
        s_pico = torch.sqrt(torch.clamp(a1[0] / N, min=0.0))
        s_pmr = torch.sqrt(torch.clamp(var, min=0.0))
        e_pmr = math.sqrt(1.0 / (2.0 * (N - 1)))      # std map of a Gaussian sample variance
        rows.append({"scale": scale, "snr_db": round(snr, 1), "sigma": sigma,
                     "nrmse_pmr_vs_pico": round(float(torch.linalg.norm(s_pmr - s_pico) / torch.linalg.norm(s_pico)), 4),
                     "mc_spread_expected": round(math.sqrt(e_pico ** 2 + e_pmr ** 2), 4),
                     "mean_std_pico": float(s_pico.mean()), "mean_std_pmr": float(s_pmr.mean()),
                     "pico_s": round(t_pico, 2), "pmr_s": round(t_pmr, 2)})
    model = (f"TV (lambda_TV {pr.extra['cs_lambda']}, {pr.extra['tv_inner']} dual steps)" if tv
             else f"L1-db4 (lambda {pr.extra['cs_lambda']})")
    return {"workload": f"CS {pr.ny}x{pr.nx}, {pr.nc} coils, {model}, FISTA {pr.extra['fista_iters']}; "
                        f"N={N} probes and {N} replicas per level",
            "levels": rows}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_init():
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"


def _cpu_worker(first_probe, nprobes):
    """One oracle process: nprobes probes of the headline workload (FP64 numpy,
    one thread); returns the seconds it took."""
    import workloads
    from oracle import pico as opico
    prob = workloads.config(2, seed=0)
    cov = opico.Covariance(opico.cartesian(prob.maps, prob.psi, prob.mask), 0.0, prob.cg_iters)
    t0 = time.perf_counter()
    opico.noise_map(cov, 11, first_probe, nprobes)
    return time.perf_counter() - t0


def cpu_baseline(per_proc=2):
    """The FP64 oracle on the host cores: one single-threaded process per core
    (at most 16, the host share of one GPU), each on its own probes of the
    headline workload; run before the GPU is touched (the pool starts fresh
    interpreters)."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    procs = max(1, min(16, ncpu))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs, initializer=_cpu_init) as pool:
        pool.starmap(_cpu_worker, [(0, 1)] * procs)            # imports and problem set-up, untimed
        t0 = time.perf_counter()
        secs = pool.starmap(_cpu_worker, [(1000 + i * per_proc, per_proc) for i in range(procs)])
        wall = time.perf_counter() - t0
    total = procs * per_proc
    return {"value": round(total / wall, 4), "unit": "probe-solves/s", "cores": procs, "kind": "oracle",
            "sample": f"{total} probes of the same 320x320 15-coil workload ({per_proc} per process), CG 30, "
                      f"FP64 numpy, {procs} single-threaded processes on {ncpu} host cores "
                      f"({wall:.1f} s wall, {sum(secs):.1f} s CPU)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-1%% leg")
    ap.add_argument("--no-ref", action="store_true", help="skip the exact reference map (implies --no-ttt)")
    ap.add_argument("--spiral-steps", type=int, default=2,
                    help="steps of the spiral Toeplitz leg (0 to skip)")
    ap.add_argument("--cs-steps", type=int, default=1,
                    help="steps of the compressed-sensing JVP leg (0 to skip)")
    ap.add_argument("--cs-tv-steps", type=int, default=1,
                    help="steps of the TV compressed-sensing JVP leg (0 to skip)")
    ap.add_argument("--serve", choices=["off", "short", "full"], default="short",
                    help="serving leg: 24 requests at 4 rates (default), 100 at 6 rates, or off")
    ap.add_argument("--cs-robustness", choices=["off", "l1wav", "tv"], default="off",
                    help="also run the CS noise-level sweep (PICO vs PMR std maps) for that model")
    ap.add_argument("--robust-n", type=int, default=3000,
                    help="probes and replicas per noise level of the CS sweep (the paper's N = 3000)")
    ap.add_argument("--no-dense", dest="dense", action="store_false",
                    help="skip the dense (matrix-core) form of the main workload")
    ap.add_argument("--no-plain", dest="plain", action="store_false",
                    help="skip the plain FP32 per-probe comparison form")
    ap.add_argument("--no-graph-leg", dest="graph_leg", action="store_false",
                    help="skip the graph-replay vs direct-launch comparison")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: the noise-map path shards by probe range "
              "across GPUs, and only the one-GPU figure is produced here (--gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline first: its process pool starts before anything touches the GPU
    progress("cpu baseline")
    cpu = None if args.no_cpu_baseline else cpu_baseline()

    import numpy as np
    import torch

    import workloads
    from paper_2605_09590_amd import pico as lib

    lib.load()
    dev = torch.device("cuda:0")
    prob = workloads.config(2, seed=0)
    ny, nx, nc = prob.ny, prob.nx, prob.nc
    K = 256
    n = ny * nx
    maps = torch.from_numpy(prob.maps.astype(np.complex64)).to(dev)
    mask = torch.from_numpy(prob.mask).to(dev)
    t0 = time.perf_counter()
    h = lib.pico_init(ny, nx, maps, prob.psi, mask, cg_iters=prob.cg_iters, probe_tile=K)
    init_s = time.perf_counter() - t0

    progress("headline workload: exact reference, time to 1 %, PMR, plain FP32, reduced grid, families")
    # exact reference map (row-unit probing of the column-separable Sigma)
    ref = torch.empty(n, dtype=torch.float64, device=dev)
    ref_s = None
    if not args.no_ref:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.pico_exact_diag(h, ref)
        torch.cuda.synchronize()
        ref_s = round(time.perf_counter() - t0, 4)

    out = {}
    # --- time to 1 % NRMSE (std map), probes in chunks of 32 with the monitor
    if not (args.no_ttt or args.no_ref):
        acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
        acc = lib.make_accum(acc_t[0], None, acc_t[1])
        chunk = 32
        curve = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_done, t_hit, n_hit = 0, None, None
        while n_done < 4096:
            lib.pico_noise_map(h, 7, n_done, chunk, 0, acc)
            n_done += chunk
            e = lib.pico_monitor_nrmse(h, acc, ref)
            t = time.perf_counter() - t0
            curve.append((n_done, round(t, 5), round(e, 5)))
            if e <= 0.01:
                t_hit, n_hit = t, n_done
                break
        out["time_to_1pct_s"] = t_hit
        out["n_at_1pct"] = n_hit
        out["nrmse_curve"] = curve[:12]

    # --- the PMR baseline on the same workload and reference: replicas in chunks
    # of 32 until the std map of the unbiased sample variance is within 1 %
    if not (args.no_ttt or args.no_ref):
        acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        acc = lib.make_accum(*acc_t)
        var = torch.empty(n, dtype=torch.float64, device=dev)
        s_ref = torch.sqrt(torch.clamp(ref, min=0.0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, hit = 0, None
        while done < 8192:
            lib.pico_pmr_baseline(h, 3, done, 32, acc)
            done += 32
            lib.pico_pmr_finalize(h, acc, var)
            e = float(torch.linalg.norm(torch.sqrt(torch.clamp(var, min=0.0)) - s_ref) / torch.linalg.norm(s_ref))
            if e <= 0.01:
                hit = (time.perf_counter() - t0, done)
                break
        out["pmr_time_to_1pct_s"] = round(hit[0], 5) if hit else None
        out["pmr_n_at_1pct"] = hit[1] if hit else None
        out["pmr_nrmse_at_stop"] = round(e, 5)

    # --- the plain FP32 per-probe form of the same estimator (comparison baseline)
    if not (args.no_ttt or args.no_ref) and args.plain:
        out["plain_fp32"] = plain_leg(torch, np, dev, prob, ref, check=(lib, h))

    # --- reduced-resolution grid (factor 2) against the same native exact map
    if not (args.no_ttt or args.no_ref):
        out["reduced_grid"] = reduced_leg(lib, torch, np, dev, prob, ref)

    # --- probe families (Sec. 2.2, Eqs. (18)-(20)): probes to a 1 % std map
    if not (args.no_ttt or args.no_ref):
        fam = {}
        for name, dist in (("random_phase", 0), ("qpsk", 1), ("rademacher", 2), ("gaussian", 3)):
            acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(2)]
            acc = lib.make_accum(acc_t[0], None, acc_t[1])
            done, n_hit, e64 = 0, None, None
            while done < 4096:
                lib.pico_noise_map(h, 41, done, 32, dist, acc)
                done += 32
                e = lib.pico_monitor_nrmse(h, acc, ref)
                if done == 64:
                    e64 = round(e, 5)
                if e <= 0.01:
                    n_hit = done
                    break
            fam[name] = {"n_at_1pct": n_hit, "nrmse_at_64": e64}
        out["probe_families"] = fam

    # --- adaptive stopping without a reference: probe tiles until the
    # standard-error proxy of the std map reaches 1 %; NRMSE vs exact reported
    if not args.no_ref:
        acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
        acc = lib.make_accum(*acc_t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        used, proxy = lib.pico_noise_map_adaptive(h, 7, 0, 4096, 0.01, 0, acc)
        t_ad = time.perf_counter() - t0
        out["adaptive_1pct"] = {"seconds": round(t_ad, 5), "probes": used, "proxy": round(proxy, 5),
                                "nrmse_vs_exact": round(lib.pico_monitor_nrmse(h, acc, ref), 5)}

    progress("headline throughput")
    # --- steady-state throughput: K=256 probes per step
    acc_t = [torch.zeros(n, dtype=torch.float64, device=dev) for _ in range(3)]
    acc = lib.make_accum(*acc_t)
    first = 0
    for _ in range(args.warmup):
        lib.pico_noise_map(h, 11, first, K, 0, acc)
        first += K
    torch.cuda.synchronize()
    lib.pico_profile_start(h)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        lib.pico_noise_map(h, 11, first, K, 0, acc)
        first += K
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    prof = lib.pico_profile_stop(h)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = K * args.steps / (gpu_ms / 1e3)
    st = lib.pico_stats_t()
    lib.pico_noise_map(h, 11, first, K, 0, acc, st)   # convergence check (outside timing)
    torch.cuda.synchronize()
    true_res = None if args.no_ref else true_residual(lib, torch, np, dev, h, prob)
    lib.pico_destroy(h)

    # --- roofline of the dominant kernel (fused p-update + normal operator)
    it_ms, it_n = prof["normal_iter"]
    avg_s = it_ms / it_n / 1e3
    flops = normal_op_flops(ny, nx, nc) * K
    bytes_alg = K * 8 * 8 * n + nc * n * 8           # x, r, p, q read and written; maps once
    achieved_tf = flops / avg_s / 1e12
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_normal_iter_cart1d_320x320x15_K256.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("kernel_src_sha") == kernel_source_digest():
            traffic = tj.get("hbm_bytes_per_launch")
    roofline = {
        "bound": "alu", "achieved": round(achieved_tf, 2), "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s", "frac": round(achieved_tf / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
        "kernel": "k_cart1d<TwoStep<20,16>, C1_ITER>", "avg_launch_us": round(avg_s * 1e6, 2),
        "flops_per_launch": flops, "alg_bytes_per_launch": bytes_alg,
        "hbm_GBs_alg": round(bytes_alg / avg_s / 1e9, 1),
    }

    progress("stream ceiling, dense forms")
    # --- the same workload with the dense per-column operator on the matrix cores
    ceiling = stream_ceiling(torch, dev)
    dense = dense_leg(lib, torch, np, dev, prob, form=2) if args.dense else None
    dense16 = dense_leg(lib, torch, np, dev, prob, form=3, ref=None if args.no_ref else ref) if args.dense else None

    progress("spiral")
    # --- second workload: spiral CG-SENSE, Toeplitz normal operator (HBM-bound path),
    # complex64 planes and the bfloat16-stream variant
    spiral = spiral_bf16 = None
    if args.spiral_steps > 0:
        spiral = spiral_leg(lib, workloads, torch, np, dev, args.spiral_steps, lib.PICO_FP32)
        spiral_bf16 = spiral_leg(lib, workloads, torch, np, dev, args.spiral_steps, lib.PICO_BF16_STREAM)

    progress("spiral R = 2, 3, 4 against exact subsets; gridding normal operator")
    spiral_ttt = spiral_grid = None
    if args.spiral_steps > 0 and not args.no_ttt:
        spiral_ttt = spiral_exact_leg(lib, workloads, torch, np, dev)
    if args.spiral_steps > 0:
        spiral_grid = spiral_gridding_leg(lib, workloads, torch, np, dev)

    progress("CS")
    # --- third workload: CS (FISTA L1-db4), batched Jacobian-vector probes
    cs_res = cs_bf16 = None
    if args.cs_steps > 0:
        cs_res = cs_leg(lib, workloads, torch, np, dev, args.cs_steps)
        cs_bf16 = cs_leg(lib, workloads, torch, np, dev, args.cs_steps, lib.PICO_BF16_STREAM)

    progress("TV-CS")
    # --- the paper's CS model: TV-regularised FISTA, Jacobian probes vs FP64 PMR replicas
    cs_tv = cs_tv_bf16 = None
    if args.cs_tv_steps > 0:
        cs_tv = cs_tv_leg(lib, workloads, torch, np, dev, args.cs_tv_steps)
        cs_tv_bf16 = cs_tv_leg(lib, workloads, torch, np, dev, args.cs_tv_steps, storage=lib.PICO_BF16_STREAM,
                               pmr=False)

    # bfloat16 storage against FP32 storage: the same probes, so the maps differ
    # by the storage rounding alone
    for leg, ref_leg in ((cs_bf16, cs_res), (cs_tv_bf16, cs_tv)):
        if leg is not None and ref_leg is not None:
            leg["map_vs_f32_storage"] = {
                "std_map_nrmse": round(std_map_nrmse(torch, leg["_map"], ref_leg["_map"]), 6),
                "var_map_rel": round(float(torch.linalg.norm(leg["_map"] - ref_leg["_map"]) /
                                           torch.linalg.norm(ref_leg["_map"])), 6),
                "probes": leg["probes_accumulated"]}
    for leg in (cs_res, cs_bf16, cs_tv, cs_tv_bf16):
        if leg is not None:
            leg.pop("_map", None)
            leg.pop("probes_accumulated", None)

    progress("CS time to converged accuracy")
    cs_conv = None
    if args.cs_steps > 0 and not args.no_ttt:
        cs_conv = {"l1wav": cs_converged_leg(lib, workloads, torch, np, dev, "l1wav", 8192)}
        if args.cs_tv_steps > 0:
            cs_conv["tv"] = cs_converged_leg(lib, workloads, torch, np, dev, "tv", 16384)

    robust = (cs_robustness(lib, workloads, torch, np, dev, N=args.robust_n, reg=args.cs_robustness)
              if args.cs_robustness != "off" else None)

    progress("serving")
    # --- serving: mixed requests under Poisson arrivals, p50 / p99 latency
    serving = None
    if args.serve != "off":
        serving = serve_leg(lib, workloads, torch, np, dev, **({"n_req": 100, "rhos": (0.25, 0.5, 0.75, 0.9, 1.1, 1.3)}
                                                                 if args.serve == "full" else {}))
    graphs = graph_leg(lib, workloads, torch, np, dev) if args.graph_leg else None

    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "probe-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cart1d 320x320 complex64, 15 coils, R=2 + 24 ACS lines, "
                               "K=256 random-phase probes per step, CG 30, FP64 dots/accumulators",
                   "probes_per_step": K, "ny": ny, "nx": nx, "coils": nc, "cg_iters": prob.cg_iters},
        **out,
        "init_s": round(init_s, 4), "reference_s": ref_s,
        "wall_s_timed": round(wall, 4),
        "cg_max_relres": st.max_relres,
        "cg_true_relres": true_res,
        "kernel_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "kernel_launches": {k: v[1] for k, v in prof.items()},
        "roofline": roofline, "cpu_baseline": cpu,
        "hbm_stream_ceiling": ceiling,
        "dense_form": dense,
        "dense_form_split_fp16": dense16,
        "spiral": spiral,
        "spiral_bf16": spiral_bf16,
        "spiral_time_to_1pct": spiral_ttt,
        "spiral_gridding_normal": spiral_grid,
        "cs": cs_res,
        "cs_bf16": cs_bf16,
        "cs_tv": cs_tv,
        "cs_tv_bf16": cs_tv_bf16,
        "cs_time_to_converged": cs_conv,
        "serving": serving,
        "graph_vs_direct": graphs,
    }
    if robust is not None:
        res["cs_robustness"] = robust
    if args.copy_calib:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calib_bytes"] = a.numel() * 8
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
