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
PICO_CGSENSE, PICO_CS_FISTA_L1WAV = range(2)
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
    ]


class pico_accum_t(ctypes.Structure):
    _fields_ = [("sum", ctypes.c_void_p), ("sum_im", ctypes.c_void_p),
                ("sumsq", ctypes.c_void_p), ("count", ctypes.c_int64)]


class pico_stats_t(ctypes.Structure):
    _fields_ = [("probes", ctypes.c_int64), ("max_relres", ctypes.c_double),
                ("mean_relres", ctypes.c_double), ("frozen", ctypes.c_int32),
                ("lambda_abs", ctypes.c_double)]


class PicoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pico status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = ["pico_init", "pico_apply_cov", "pico_apply_jvp", "pico_recon", "pico_noise_map", "pico_finalize",
           "pico_pmr_baseline", "pico_pmr_finalize", "pico_monitor_nrmse", "pico_exact_diag",
           "pico_profile_start", "pico_profile_stop", "pico_lambda_abs", "pico_destroy",
           "pico_last_error"]
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
    lib.pico_apply_cov.argtypes = [vp, vp, vp, i32, vp]
    lib.pico_apply_jvp.argtypes = [vp, vp, vp, i32, vp]
    lib.pico_recon.argtypes = [vp, vp, vp]
    lib.pico_noise_map.argtypes = [vp, u64, i64, i64, i32, ctypes.POINTER(pico_accum_t),
                                   ctypes.POINTER(pico_stats_t), vp]
    lib.pico_finalize.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp, vp]
    lib.pico_pmr_baseline.argtypes = [vp, u64, i64, i64, ctypes.POINTER(pico_accum_t),
                                      ctypes.POINTER(pico_stats_t), vp]
    lib.pico_pmr_finalize.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp, vp]
    lib.pico_monitor_nrmse.argtypes = [vp, ctypes.POINTER(pico_accum_t), vp,
                                       ctypes.POINTER(ctypes.c_double), vp]
    lib.pico_exact_diag.argtypes = [vp, vp, vp]
    lib.pico_profile_start.argtypes = [vp]
    lib.pico_profile_stop.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    lib.pico_lambda_abs.argtypes = [vp]
    lib.pico_lambda_abs.restype = ctypes.c_double
    lib.pico_destroy.argtypes = [vp]
    lib.pico_destroy.restype = None
    lib.pico_last_error.argtypes = []
    lib.pico_last_error.restype = ctypes.c_char_p
    for name in ("pico_init", "pico_apply_cov", "pico_apply_jvp", "pico_recon", "pico_noise_map", "pico_finalize",
                 "pico_pmr_baseline", "pico_pmr_finalize", "pico_monitor_nrmse",
                 "pico_exact_diag", "pico_profile_start", "pico_profile_stop"):
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


def pico_last_error() -> str:
    return load().pico_last_error().decode()


def pico_init(ny, nx, maps, psi, mask, sampling=PICO_CART_1D, lam=0.0, cg_iters=30, cg_tol=0.0,
              power_iters=15, power_margin=1.01, probe_tile=256, recon=PICO_CGSENSE,
              traj=None, nsamples=0, kdata=None, fista_iters=100, cs_lambda=1e-3,
              wavelet_levels=4, stream=None):
    """pico_init: ``maps`` complex64 device tensor [nc][ny][nx]; ``psi`` numpy
    complex128 [nc][nc] or None; ``mask`` uint8 device tensor.  Returns the handle."""
    lib = load()
    d = pico_op_desc_t()
    d.ny, d.nx, d.ncoils = int(ny), int(nx), int(maps.shape[0])
    d.maps = maps.data_ptr()
    keep = None
    if psi is not None:
        keep = np.ascontiguousarray(np.asarray(psi, np.complex128)).view(np.float64)
        d.psi = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.sampling = sampling
    d.mask = mask.data_ptr() if mask is not None else None
    d.traj = traj.data_ptr() if traj is not None else None
    d.nsamples = nsamples
    d.lambda_ = lam
    d.cg_iters = cg_iters
    d.cg_tol = cg_tol
    d.power_iters = power_iters
    d.power_margin = power_margin
    d.probe_tile = probe_tile
    d.recon = recon
    d.kdata = kdata.data_ptr() if kdata is not None else None
    d.fista_iters = fista_iters
    d.cs_lambda = cs_lambda
    d.wavelet_levels = wavelet_levels
    h = ctypes.c_void_p()
    _check(lib.pico_init(ctypes.byref(d), _stream(stream), ctypes.byref(h)))
    del keep
    return h


def pico_apply_cov(h, v, u, k, stream=None):
    return _check(load().pico_apply_cov(h, _ptr(v), _ptr(u), int(k), _stream(stream)))


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


def pico_pmr_finalize(h, acc, var, stream=None):
    return _check(load().pico_pmr_finalize(h, ctypes.byref(acc), _ptr(var), _stream(stream)))


def pico_monitor_nrmse(h, acc, ref_var, stream=None) -> float:
    out = ctypes.c_double()
    _check(load().pico_monitor_nrmse(h, ctypes.byref(acc), _ptr(ref_var), ctypes.byref(out),
                                     _stream(stream)))
    return out.value


def pico_exact_diag(h, var, stream=None):
    return _check(load().pico_exact_diag(h, _ptr(var), _stream(stream)))


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
