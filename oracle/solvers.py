"""Conjugate gradients and power method, FP64 (oracle side).

CG on the normal equations (A^H A + lam I) x = A^H b_w is the CG-SENSE
solver of Sec. 2.1, Eq. (6) (Pruessmann et al. 2001).  The paper runs it for
a fixed number of iterations (Sec. 3.2.1: 25) or to a relative tolerance
(Sec. 3.2.2: tol 1e-2, at most 100); PICO reuses it for every probe
(Sec. 2.2, "Implicit matrix-vector product via CG"; App. A, Algorithm 1).

Readings where the paper is silent: x0 = 0; the step length uses
Re(p^H q) (the operator is Hermitian, so the imaginary part is rounding);
tolerance mode stops a right-hand side once ||r|| / ||r0|| <= tol; a
breakdown (p^H q <= 0, or a non-finite scalar) freezes that right-hand side.

Spectral normalisation: lambda_max of M by a 15-step power method with a
1.01 safety margin, applied to every forward operator (Sec. 3.2.1, 3.3).
"""
from __future__ import annotations

import numpy as np

from . import philox


def cg(apply, b, iters: int, lam: float = 0.0, tol: float = 0.0, return_info=False):
    """Hestenes-Stiefel CG for (M + lam I) x = b, x0 = 0.

    ``apply(p)`` returns M p.  Returns x (and an info dict when asked:
    final relative residual, iterations taken, frozen flag).
    """
    b = np.asarray(b, np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    rr0 = rr
    frozen = False
    done = 0
    for _ in range(iters):
        if rr == 0.0:
            break
        q = apply(p) + lam * p
        pq = np.vdot(p, q).real
        if not (pq > 0.0) or not np.isfinite(pq):
            frozen = True
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        done += 1
        if tol > 0.0 and np.sqrt(rr_new / rr0) <= tol:
            rr = rr_new
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    if return_info:
        return x, {"relres": float(np.sqrt(rr / rr0)) if rr0 > 0 else 0.0,
                   "iters": done, "frozen": frozen}
    return x


def power_method(apply, shape, iters: int = 15, margin: float = 1.01):
    """Largest eigenvalue of the Hermitian PSD operator, times ``margin``.

    Start vector: a unit random-phase vector from the Philox stream reserved
    for it (key 0, draw 0).  Each step: w = M v, Rayleigh quotient
    Re(v^H w), v = w / ||w||.  Returns margin * (last Rayleigh quotient).
    """
    n = int(np.prod(shape))
    v = philox.probe(0, 0, n, "phase", stream=philox.STREAM_POWER).reshape(shape)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = apply(v)
        lam = np.vdot(v, w).real
        v = w / np.linalg.norm(w)
    return margin * lam
