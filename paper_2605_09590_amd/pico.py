"""Thin Python binding of libpico (include/pico.h), argument marshalling only.

Every function has the C name and forwards to the shared library; device
buffers are torch tensors on the ROCm device (their ``data_ptr()`` is passed),
streams are torch streams.  There is no fallback: if libpico.so is missing or
fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpico.so")

PICO_OK, PICO_EINVAL, PICO_ENOMEM, PICO_EDEVICE, PICO_EUNSUPPORTED, PICO_ENOTCONV = range(6)
PICO_CART_1D, PICO_CART_2D, PICO_NONCART = range(3)
PICO_CGSENSE, PICO_CS_FISTA_L1WAV, PICO_CS_FISTA_TV = range(3)
PICO_FP32, PICO_BF16_MAPS, PICO_BF16_STREAM = range(3)
PROBES = {"phase": 0, "qpsk": 1, "rademacher": 2, "gaussian": 3}


class pico_op_desc_t(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("ncoils", ctypes.c_int32),
        ("maps", ctypes.c_void_p),
        ("psi", ctypes.POINTER(ctypes.c_double)),
        ("sampling", ctypes.c_int32),
        ("mask", ctypes.c_void_p),
        ("traj", ctypes.c_void_p),
        ("nsamples", ctypes.c_int64),
        ("lambda_", ctypes.c_double),
        ("cg_iters", ctypes.c_int32),
        ("cg_tol", ctypes.c_double),
        ("power_iters", ctypes.c_int32),
        ("power_margin", ctypes.c_double),
        ("probe_tile", ctypes.c_int32),
        ("recon", ctypes.c_int32),
        ("kdata", ctypes.c_void_p),
        ("fista_iters", ctypes.c_int32),
        ("cs_lambda", ctypes.c_double),
        ("wavelet_levels", ctypes.c_int32),
        ("oversamp", ctypes.c_double),
        ("kb_width", ctypes.c_int32),
        ("normal_form", ctypes.c_int32),
        ("tv_inner_iters", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("noncart_normal", ctypes.c_int32),
    ]


class pico_accum_t(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_void_p), ("sum_im", ctypes.c_void_p),
                ("sumsq", ctypes.c_void_p), ("count", ctypes.c_int64)]


class pico_stats_t(ctypes.Structure):
    _fields_ = [("probes", ctypes.c_int64), ("max_relres", ctypes.c_double),
                ("mean_relres", ctypes.c_double), ("frozen", ctypes.c_int32),
                ("lambda_abs", ctypes.c_double)]


class pico_request_info_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("first_probe", ctypes.c_int64), ("probes", ctypes.c_int64),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double),
                ("bytes_peak", ctypes.c_uint64), ("bytes_resident", ctypes.c_uint64),
                ("probe_tile", ctypes.c_int32), ("op_reused", ctypes.c_int32),
                ("error", ctypes.c_char * 160)]


class pico_tune_t(ctypes.Structure):
    _fields_ = [("probe_tile", ctypes.c_int32), ("normal_form", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("probes_per_s", ctypes.c_double), ("from_cache", ctypes.c_int32)]


class PicoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pico status {status}: {msg}")
        self.status = status


_lib = None

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocator_keep = None     # the installed callback objects (ctypes needs them alive)

EXPORTS = ["pico_init", "pico_apply_cov", "pico_apply_jvp", "pico_apply_nufft", "pico_recon", "pico_noise_map", "pico_finalize",
           "pico_pmr_baseline", "pico_pmr_finalize", "pico_pmr_cs", "pico_monitor_nrmse", "pico_monitor_stderr", "pico_noise_map_adaptive", "pico_exact_diag",
           "pico_init_reduced", "pico_upsample_map",
           "pico_profile_start", "pico_profile_stop", "pico_lambda_abs", "pico_destroy",
           "pico_last_error", "pico_estimate_bytes", "pico_op_bytes", "pico_server_create",
           "pico_server_submit", "pico_server_poll", "pico_server_wait_idle", "pico_server_usage",
           "pico_server_destroy", "pico_set_allocator", "pico_pmr_cs_noalloc", "pico_autotune",
           "pico_server_set_tuning", "pico_server_cache_stats"]
PROF_KINDS = 8
PROF_NAMES = ["normal_first", "normal_iter", "cg_update", "cg_scalars", "accumulate", "other"]


def load(path: str = LIB_PATH):
    """Load libpico.so (torch first, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.pico_init.argtypes = [ctypes.POINTER(pico_op_desc_t), vp, ctypes.POINTER(vp)]
    lib.pico_init_reduced.argtypes = [ctypes.POINTER(pico_op_desc_t), i32, vp, ctypes.POINTER(vp)]
    lib.pico_upsample_map.argtypes = [vp, vp, vp, vp]
    lib.pico_apply_cov.argtypes = [vp, vp, vp, i32, vp]
    lib.pico_apply_jvp.argtypes = [vp, vp, vp, i32, vp]
    lib.pico_apply_nufft.argtypes = [vp, i32, vp, vp, i32, vp]
    lib.pico_recon.argtypes = [vp, vp, vp]
    lib.pico_noise_map.argtypes = [vp, u64, i64, i64, i32, ctypes.POINTER(pico_accum_t),
                                   ctypes.POINTER(pico_stats_t), vp]
    lib.pico_finalize.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp, vp]
    lib.pico_pmr_baseline.argtypes = [vp, u64, i64, i64, ctypes.POINTER(pico_accum_t),
                                      ctypes.POINTER(pico_stats_t), vp]
    lib.pico_pmr_finalize.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp, vp]
    lib.pico_pmr_cs.argtypes = [vp, u64, i64, i64, ctypes.c_double, ctypes.POINTER(pico_accum_t), vp]
    lib.pico_pmr_cs_noalloc.argtypes = [vp, u64, i64, i64, ctypes.c_double, ctypes.POINTER(pico_accum_t), vp]
    lib.pico_monitor_nrmse.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp,
                                       ctypes.POINTER(ctypes.c_double), vp]
    lib.pico_exact_diag.argtypes = [vp, vp, vp]
    lib.pico_monitor_stderr.argtypes = [vp, ctypes.POINTER(pico_accum_t), ctypes.POINTER(ctypes.c_double), vp]
    lib.pico_noise_map_adaptive.argtypes = [vp, u64, i64, i64, ctypes.c_double, i32, ctypes.POINTER(pico_accum_t),
                                            ctypes.POINTER(pico_stats_t), ctypes.POINTER(i64),
                                            ctypes.POINTER(ctypes.c_double), vp]
    lib.pico_profile_start.argtypes = [vp]
    lib.pico_profile_stop.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.pico_lambda_abs.argtypes = [vp]
    lib.pico_lambda_abs.restype = ctypes.c_double
    lib.pico_destroy.argtypes = [vp]
    lib.pico_destroy.restype = None
    lib.pico_last_error.argtypes = []
    lib.pico_last_error.restype = ctypes.c_char_p
    lib.pico_estimate_bytes.argtypes = [ctypes.POINTER(pico_op_desc_t), ctypes.POINTER(u64),
                                        ctypes.POINTER(u64)]
    lib.pico_op_bytes.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.pico_server_create.argtypes = [u64, i32, i32, ctypes.POINTER(vp)]
    lib.pico_server_submit.argtypes = [vp, ctypes.POINTER(pico_op_desc_t), u64, i64, i64, i32,
                                       ctypes.POINTER(pico_accum_t), ctypes.POINTER(u64)]
    lib.pico_server_poll.argtypes = [vp, ctypes.POINTER(pico_request_info_t), i32,
                                     ctypes.POINTER(i32)]
    lib.pico_server_wait_idle.argtypes = [vp, ctypes.c_double]
    lib.pico_server_usage.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                      ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pico_server_destroy.argtypes = [vp]
    lib.pico_server_destroy.restype = None
    lib.pico_set_allocator.argtypes = [ALLOC_FN, FREE_FN, vp]
    lib.pico_autotune.argtypes = [ctypes.POINTER(pico_op_desc_t), u64, ctypes.c_char_p, vp,
                                  ctypes.POINTER(pico_tune_t)]
    lib.pico_server_set_tuning.argtypes = [vp, ctypes.c_char_p]
    lib.pico_server_cache_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(u64), ctypes.POINTER(i64),
                                            ctypes.POINTER(i64)]
    for name in ("pico_init", "pico_apply_cov", "pico_apply_jvp", "pico_apply_nufft", "pico_recon", "pico_noise_map", "pico_finalize",
                 "pico_pmr_baseline", "pico_pmr_finalize", "pico_pmr_cs", "pico_pmr_cs_noalloc",
                 "pico_monitor_nrmse", "pico_exact_diag", "pico_profile_start", "pico_profile_stop",
                 "pico_monitor_stderr", "pico_noise_map_adaptive",
                 "pico_estimate_bytes", "pico_op_bytes", "pico_server_create", "pico_server_submit",
                 "pico_server_poll", "pico_server_wait_idle", "pico_server_usage", "pico_set_allocator",
                 "pico_autotune", "pico_server_set_tuning", "pico_server_cache_stats"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st):
    if st != PICO_OK:
        raise PicoError(st, _lib.pico_last_error().decode())
    return st


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def pico_set_allocator(alloc=None, free=None, ctx=None):
    """pico_set_allocator with Python callables alloc(nbytes) -> int address
    (0 on failure) and free(address); both None restores hipMalloc / hipFree."""
    global _allocator_keep
    lib = load()
    if alloc is None and free is None:
        _check(lib.pico_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator_keep = None
        return
    a = ALLOC_FN(lambda nbytes, _ctx: alloc(int(nbytes)) or None)
    f = FREE_FN(lambda ptr, _ctx: free(int(ptr)))
    _check(lib.pico_set_allocator(a, f, ctx))
    _allocator_keep = (a, f)


def use_torch_allocator(enable: bool = True):
    """Route every library workspace through torch's caching allocator
    (torch.cuda.caching_allocator_alloc / _delete on the current device and
    stream), or back to hipMalloc / hipFree."""
    if not enable:
        return pico_set_allocator()
    import torch

    def alloc(nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(nbytes)
        except RuntimeError:     # out of memory: the library reports PICO_ENOMEM
            return 0

    pico_set_allocator(alloc, torch.cuda.caching_allocator_delete)


def pico_last_error() -> str:
    return load().pico_last_error().decode()


def _addr(x):
    """Device address of a tensor (``data_ptr()``), an int address, or None."""
    if x is None:
        return None
    return int(x) if isinstance(x, int) else x.data_ptr()


def make_desc(ny, nx, maps, psi, mask, sampling=PICO_CART_1D, lam=0.0, cg_iters=30, cg_tol=0.0,
              power_iters=15, power_margin=1.01, probe_tile=256, recon=PICO_CGSENSE,
              traj=None, nsamples=0, kdata=None, fista_iters=100, cs_lambda=1e-3,
              wavelet_levels=4, oversamp=2.0, kb_width=0, normal_form=0, ncoils=None,
              tv_inner_iters=10, storage=0, graph=0, noncart_normal=0):
    """pico_op_desc_t for the arguments of pico_init; returns (desc, keep) where
    ``keep`` holds the host psi array the descriptor points to."""
    d = pico_op_desc_t()
    d.ny, d.nx = int(ny), int(nx)
    d.ncoils = int(ncoils if ncoils is not None else maps.shape[0])
    d.maps = _addr(maps)
    keep = None
    if psi is not None:
        keep = np.ascontiguousarray(np.asarray(psi, np.complex128)).view(np.float64)
        d.psi = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.sampling = sampling
    d.mask = _addr(mask)
    d.traj = _addr(traj)
    d.nsamples = nsamples
    d.lambda_ = lam
    d.cg_iters = cg_iters
    d.cg_tol = cg_tol
    d.power_iters = power_iters
    d.power_margin = power_margin
    d.probe_tile = probe_tile
    d.recon = recon
    d.kdata = _addr(kdata)
    d.fista_iters = fista_iters
    d.cs_lambda = cs_lambda
    d.wavelet_levels = wavelet_levels
    d.oversamp = oversamp
    d.kb_width = kb_width
    d.normal_form = normal_form
    d.tv_inner_iters = tv_inner_iters
    d.storage = storage
    d.graph = graph
    d.noncart_normal = noncart_normal
    return d, keep


def pico_init(ny, nx, maps, psi, mask, sampling=PICO_CART_1D, lam=0.0, cg_iters=30, cg_tol=0.0,
              power_iters=15, power_margin=1.01, probe_tile=256, recon=PICO_CGSENSE,
              traj=None, nsamples=0, kdata=None, fista_iters=100, cs_lambda=1e-3,
              wavelet_levels=4, oversamp=2.0, kb_width=0, normal_form=0, stream=None,
              tv_inner_iters=10, storage=0, graph=0, noncart_normal=0):
    """pico_init: ``maps`` complex64 device tensor [nc][ny][nx]; ``psi`` numpy
    complex128 [nc][nc] or None; ``mask`` uint8 device tensor.  Returns the handle."""
    lib = load()
    d, keep = make_desc(ny, nx, maps, psi, mask, sampling, lam, cg_iters, cg_tol, power_iters,
                        power_margin, probe_tile, recon, traj, nsamples, kdata, fista_iters,
                        cs_lambda, wavelet_levels, oversamp, kb_width, normal_form,
                        tv_inner_iters=tv_inner_iters, storage=storage, graph=graph,
                        noncart_normal=noncart_normal)
    h = ctypes.c_void_p()
    _check(lib.pico_init(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
    del keep
    return h


def pico_estimate_bytes(desc):
    """(resident, peak) device bytes pico_init takes for ``desc`` (host only)."""
    r, p = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().pico_estimate_bytes(ctypes.byref(desc), ctypes.byref(r), ctypes.byref(p)))
    return r.value, p.value


def pico_op_bytes(h):
    r, p = ctypes.c_uint64(), ctypes.c_uint64()
    _check(load().pico_op_bytes(h, ctypes.byref(r), ctypes.byref(p)))
    return r.value, p.value


def pico_apply_cov(h, v, u, k, stream=None):
    return _check(load().pico_apply_cov(h, _ptr(v), _ptr(u), int(k), _stream(stream)))


def pico_apply_nufft(h, adjoint, x, out, k, stream=None):
    return _check(load().pico_apply_nufft(h, int(adjoint), _ptr(x), _ptr(out), int(k), _stream(stream)))


def pico_apply_jvp(h, w, u, k, stream=None):
    return _check(load().pico_apply_jvp(h, _ptr(w), _ptr(u), int(k), _stream(stream)))


def pico_recon(h, x, stream=None):
    return _check(load().pico_recon(h, _ptr(x), _stream(stream)))


def make_accum(sum_, sum_im=None, sumsq=None, count=0):
    return pico_accum_t(sum_.data_ptr(), None if sum_im is None else sum_im.data_ptr(),
                        None if sumsq is None else sumsq.data_ptr(), count)


def pico_noise_map(h, seed, first_probe, nprobes, dist, acc, stats=None, stream=None):
    return _check(load().pico_noise_map(h, int(seed), int(first_probe), int(nprobes), int(dist),
                                        ctypes.byref(acc),
                                        None if stats is None else ctypes.byref(stats),
                                        _stream(stream)))


def pico_finalize(h, acc, var, stream=None):
    return _check(load().pico_finalize(h, ctypes.byref(acc), _ptr(var), _stream(stream)))


def pico_pmr_baseline(h, seed, first, nrep, acc, stats=None, stream=None):
    return _check(load().pico_pmr_baseline(h, int(seed), int(first), int(nrep), ctypes.byref(acc),
                                           None if stats is None else ctypes.byref(stats),
                                           _stream(stream)))


def pico_pmr_cs(h, seed, first, nrep, sigma, acc, stream=None):
    return _check(load().pico_pmr_cs(h, int(seed), int(first), int(nrep), float(sigma), ctypes.byref(acc),
                                     _stream(stream)))


def pico_pmr_cs_noalloc(h, seed, first, nrep, sigma, acc, stream=None):
    return _check(load().pico_pmr_cs_noalloc(h, int(seed), int(first), int(nrep), float(sigma),
                                             ctypes.byref(acc), _stream(stream)))


def pico_pmr_finalize(h, acc, var, stream=None):
    return _check(load().pico_pmr_finalize(h, ctypes.byref(acc), _ptr(var), _stream(stream)))


def pico_monitor_nrmse(h, acc, ref_var, stream=None) -> float:
    out = ctypes.c_double()
    _check(load().pico_monitor_nrmse(h, ctypes.byref(acc), _ptr(ref_var), ctypes.byref(out),
                                     _stream(stream)))
    return out.value


def pico_monitor_stderr(h, acc, stream=None) -> float:
    v = ctypes.c_double()
    _check(load().pico_monitor_stderr(h, ctypes.byref(acc), ctypes.byref(v), _stream(stream)))
    return v.value


def pico_noise_map_adaptive(h, seed, first_probe, max_probes, target, dist, acc, stats=None, stream=None):
    """Returns (probes used, final proxy)."""
    used, px = ctypes.c_int64(), ctypes.c_double()
    _check(load().pico_noise_map_adaptive(h, int(seed), int(first_probe), int(max_probes), float(target),
                                          int(dist), ctypes.byref(acc),
                                          ctypes.byref(stats) if stats is not None else None,
                                          ctypes.byref(used), ctypes.byref(px), _stream(stream)))
    return used.value, px.value


def pico_exact_diag(h, var, stream=None):
    return _check(load().pico_exact_diag(h, _ptr(var), _stream(stream)))


def pico_init_reduced(factor, ny, nx, maps, psi, mask, stream=None, **kw):
    """pico_init_reduced: the coarse operator of factor ``factor`` for the
    native problem described by the arguments of pico_init (native ny, nx,
    maps, mask or trajectory).  Returns the handle of the coarse operator."""
    lib = load()
    d, keep = make_desc(ny, nx, maps, psi, mask, **kw)
    h = ctypes.c_void_p()
    _check(lib.pico_init_reduced(ctypes.byref(d), int(factor), _stream(stream), ctypes.byref(h)))
    del keep
    return h


def pico_upsample_map(h, coarse, var, stream=None):
    """Native map ``var`` from the coarse map of a reduced operator."""
    return _check(load().pico_upsample_map(h, _ptr(coarse), _ptr(var), _stream(stream)))


def pico_profile_start(h):
    return _check(load().pico_profile_start(h))


def pico_profile_stop(h):
    """Returns {kind name: (total ms, launches)}."""
    ms = (ctypes.c_double * PROF_KINDS)()
    n = (ctypes.c_int64 * PROF_KINDS)()
    _check(load().pico_profile_stop(h, ms, n))
    return {PROF_NAMES[k]: (ms[k], n[k]) for k in range(len(PROF_NAMES))}


def pico_lambda_abs(h) -> float:
    return load().pico_lambda_abs(h)


def pico_destroy(h) -> None:
    load().pico_destroy(h)


def pico_server_create(hbm_budget, max_slots=4, tiles_in_flight=2):
    h = ctypes.c_void_p()
    _check(load().pico_server_create(int(hbm_budget), int(max_slots), int(tiles_in_flight),
                                     ctypes.byref(h)))
    return h


def pico_server_submit(srv, desc, seed, first_probe, nprobes, dist, acc) -> int:
    rid = ctypes.c_uint64()
    _check(load().pico_server_submit(srv, ctypes.byref(desc), int(seed), int(first_probe),
                                     int(nprobes), int(dist), ctypes.byref(acc), ctypes.byref(rid)))
    return rid.value


def pico_server_poll(srv, max_n=256):
    """Finished requests, oldest first, as dicts of pico_request_info_t fields."""
    arr = (pico_request_info_t * max_n)()
    n = ctypes.c_int32()
    _check(load().pico_server_poll(srv, arr, max_n, ctypes.byref(n)))
    out = []
    for i in range(n.value):
        r = arr[i]
        out.append({"id": r.id, "status": r.status, "first_probe": r.first_probe,
                    "probes": r.probes, "t_submit_ms": r.t_submit_ms,
                    "t_admit_ms": r.t_admit_ms, "t_done_ms": r.t_done_ms,
                    "bytes_peak": r.bytes_peak, "bytes_resident": r.bytes_resident,
                    "probe_tile": r.probe_tile, "op_reused": r.op_reused,
                    "error": r.error.decode(errors="replace")})
    return out


def pico_server_wait_idle(srv, timeout_s=-1.0):
    return _check(load().pico_server_wait_idle(srv, float(timeout_s)))


def pico_server_usage(srv):
    b, u = ctypes.c_uint64(), ctypes.c_uint64()
    q, a = ctypes.c_int32(), ctypes.c_int32()
    _check(load().pico_server_usage(srv, ctypes.byref(b), ctypes.byref(u), ctypes.byref(q),
                                    ctypes.byref(a)))
    return {"budget": b.value, "arena_used": u.value, "queued": q.value, "active": a.value}


def pico_autotune(desc, max_bytes=0, cache_path=None, stream=None):
    """pico_autotune: returns dict(probe_tile, normal_form, graph, probes_per_s, from_cache)."""
    t = pico_tune_t()
    _check(load().pico_autotune(ctypes.byref(desc), int(max_bytes),
                                None if cache_path is None else os.fsencode(cache_path), _stream(stream),
                                ctypes.byref(t)))
    return {"probe_tile": t.probe_tile, "normal_form": t.normal_form, "graph": t.graph,
            "probes_per_s": t.probes_per_s, "from_cache": bool(t.from_cache)}


def pico_server_set_tuning(srv, cache_path):
    return _check(load().pico_server_set_tuning(srv, None if cache_path is None else os.fsencode(cache_path)))


def pico_server_cache_stats(srv):
    n, b, h, m = ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().pico_server_cache_stats(srv, ctypes.byref(n), ctypes.byref(b), ctypes.byref(h), ctypes.byref(m)))
    return {"resident_ops": n.value, "resident_bytes": b.value, "hits": h.value, "misses": m.value}


def pico_server_destroy(srv) -> None:
    load().pico_server_destroy(srv)


class Server:
    """Owner of a pico_server_t.  ``submit`` takes the pico_init arguments plus
    the probe range and an accumulator; the tensors it is given stay referenced
    here until ``poll`` has reported the request."""

    def __init__(self, hbm_budget, max_slots=4, tiles_in_flight=2):
        self.h = pico_server_create(hbm_budget, max_slots, tiles_in_flight)
        self._keep = {}

    def submit(self, seed, first_probe, nprobes, acc, dist=0, **desc_kw):
        d, keep = make_desc(**desc_kw)
        rid = pico_server_submit(self.h, d, seed, first_probe, nprobes, dist, acc)
        self._keep[rid] = (desc_kw, acc, keep)
        return rid

    def poll(self, max_n=256):
        out = pico_server_poll(self.h, max_n)
        for r in out:
            self._keep.pop(r["id"], None)
        return out

    def wait_idle(self, timeout_s=-1.0):
        return pico_server_wait_idle(self.h, timeout_s)

    def usage(self):
        return pico_server_usage(self.h)

    def set_tuning(self, cache_path):
        return pico_server_set_tuning(self.h, cache_path)

    def cache_stats(self):
        return pico_server_cache_stats(self.h)

    def close(self):
        if self.h:
            pico_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
