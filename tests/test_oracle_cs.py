"""Pins of the oracle's wavelet transform, FISTA map and its Jacobian probes.

  * db4 derived by spectral factorisation: unit DC gain sqrt(2), double-shift
    orthonormality, 4 vanishing moments of the high-pass filter;
    the 2-D transform is orthonormal (norm preserving, inverse = adjoint);
    a constant image has no detail energy.
  * Forward-mode Jacobian of the FISTA map vs central finite differences of
    the map itself (the map is piecewise linear in b).
  * lam = 0: FISTA is linear in b, so J w equals the map applied to w.
  * lam = 0 and many iterations: E|J w|^2 over an exact probe enumeration
    tends to diag(M^-1) (the least-squares covariance, Sec. 2.1 Eq. (9)).
  * db4 taps equal the published table (Daubechies, Ten Lectures, Table 6.1;
    tests/golden/db4_taps.txt), which fixes the spectral-factorisation root
    choice the filter identities leave open.
  * FISTA at lam > 0 solves the stated problem: after many iterations the
    L1-db4 iterate meets the first-order optimality conditions of
    1/2 ||A x - b||^2 / s^2 + lam ||(Psi x)_detail||_1, and the TV iterate is
    a fixed point of the exact proximal-gradient map (the prox by an
    independent solver); the objective gap obeys Beck and Teboulle's
    O(1/k^2) bound (SIAM J. Imaging Sci. 2009, Thm. 4.4) at every k; the
    momentum weights start at 0 and follow Nesterov's sequence.
"""
import os
import itertools

import numpy as np

import workloads
from oracle import cs, pico, sense, wavelet


def test_db4_filter_properties():
    h, g = wavelet.wavelet_filter(4)
    assert h.size == 8
    assert abs(h.sum() - np.sqrt(2)) < 1e-14
    for m in range(4):
        v = np.dot(h[: 8 - 2 * m], h[2 * m:])
        assert abs(v - (1.0 if m == 0 else 0.0)) < 1e-14
    k = np.arange(8)
    for m in range(4):
        assert abs(np.sum(g * k ** m)) < 1e-10
    assert abs(np.sum(g * k ** 4)) > 1.0


def test_wavelet_2d_orthonormal_and_constant_image():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((64, 48)) + 1j * rng.standard_normal((64, 48))
    c = wavelet.wavedec2(x, 3)
    assert abs(np.linalg.norm(c) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.abs(wavelet.waverec2(c, 3) - x).max() < 1e-12
    y = rng.standard_normal((64, 48))
    assert abs(np.vdot(wavelet.wavedec2(y, 3), c) - np.vdot(y, x)) < 1e-10
    cc = wavelet.wavedec2(np.full((32, 32), 2.0), 2)
    m = wavelet.detail_mask((32, 32), 2)
    assert np.abs(cc[m]).max() < 1e-12


def _cs_problem(n=32, nc=2, seed=3, lam=2e-3, iters=12):
    rng = np.random.default_rng(seed)
    maps = workloads.coil_maps(n, n, nc, rng)
    psi = workloads.noise_cov(nc, rng)
    mask = workloads.poisson_disc_mask(n, n, 2.0, 6, seed=seed)
    op = pico.cartesian(maps, psi, mask)
    x = workloads.phantom(n, rng)
    b = op.forward(x)
    b = b + 0.01 * op.P[None] * (rng.standard_normal(b.shape) + 1j * rng.standard_normal(b.shape))
    return op, b, cs.FistaL1Wavelet(op, lam, iters, levels=2)


def test_jvp_matches_central_differences():
    op, b, f = _cs_problem()
    _, coeffs = f.recon(b, store=True)
    w = cs.kspace_probe(op, 4, 0)
    jw = f.jvp(w, coeffs)
    # small enough that no coefficient crosses the threshold kink
    eps = 1e-9
    fd = (f.recon(b + eps * w) - f.recon(b - eps * w)) / (2 * eps)
    assert np.linalg.norm(jw - fd) < 1e-5 * np.linalg.norm(fd)
    # and the soft-threshold derivative on its own
    rng = np.random.default_rng(1)
    c = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    dc = rng.standard_normal(500) + 1j * rng.standard_normal(500)
    m = np.ones(500, bool)
    num = (cs.soft(c + 1e-7 * dc, 0.8, m) - cs.soft(c - 1e-7 * dc, 0.8, m)) / 2e-7
    assert np.abs(cs.dsoft(c, dc, 0.8, m) - num).max() < 1e-6


def test_lambda_zero_is_linear():
    op, b, f = _cs_problem(lam=0.0)
    _, coeffs = f.recon(b, store=True)
    w = cs.kspace_probe(op, 4, 1)
    assert np.linalg.norm(f.jvp(w, coeffs) - f.recon(w)) < 1e-12 * np.linalg.norm(f.recon(w))


def test_lambda_zero_long_run_gives_least_squares_variance():
    # full Cartesian sampling of a 2-coil 4x2 system: for lam = 0 the FISTA map
    # tends to M^-1 A^H, so diag(J J^H) (by unit k-space probes) -> diag(M^-1)
    rng = np.random.default_rng(2)
    maps = workloads.coil_maps(4, 2, 2, rng)
    psi = workloads.noise_cov(2, rng)
    op = pico.cartesian(maps, psi, np.ones(4, np.uint8))
    f = cs.FistaL1Wavelet(op, 0.0, 300, levels=1)
    _, coeffs = f.recon(np.zeros((2, 4, 2), np.complex128), store=True)
    exact = np.real(np.diag(np.linalg.inv(op.dense_normal()))).reshape(4, 2)
    JJ = np.zeros((4, 2))
    for j in range(16):
        e = np.zeros(16, np.complex128)
        e[j] = 1.0
        JJ += np.abs(f.jvp(e.reshape(2, 4, 2), coeffs)) ** 2
    assert np.allclose(JJ, exact, rtol=1e-6)


def test_pmr_cs_replicas_are_difference_quotients():
    # lam = 0: the FISTA map is linear, so every replica's (x_r - x_0) / sigma is
    # the reconstruction of the noise itself, for any sigma
    op, b, f = _cs_problem(lam=0.0)
    acc = cs.pmr_cs(f, b, 7, 0, 3, sigma=0.37)
    ref = sum(f.recon(pico.pmr_noise(op, 7, r)) for r in range(3))
    assert np.linalg.norm(acc["sum"] + 1j * acc["sum_im"] - ref) < 1e-10 * np.linalg.norm(ref)
    # lam > 0, tiny sigma: each replica is the Jacobian applied to its noise
    # (first order; the step stays off the threshold kinks)
    op, b, f = _cs_problem()
    x0, coeffs = f.recon(b, store=True)
    for r in range(2):
        a = cs.pmr_cs(f, b, 9, r, 1, sigma=1e-9, x0=x0)
        jn = f.jvp(pico.pmr_noise(op, 9, r), coeffs)
        assert np.linalg.norm(a["sum"] + 1j * a["sum_im"] - jn) < 1e-5 * np.linalg.norm(jn)
        assert np.allclose(a["sumsq"], np.abs(jn) ** 2, rtol=1e-4, atol=1e-8 * np.abs(jn).max() ** 2)


# ---------------------------------------------------------------- TV model
def _chambolle_prox(z, lam, iters=4000, tau=0.125):
    """Chambolle's projection algorithm (J. Math. Imaging Vis. 2004), written
    independently of the oracle: p <- (p + tau g) / (1 + tau |g|) with
    g = grad(div p - z / lam), div p = -(D^H p); prox = z - lam div p."""
    def grad(x):
        return np.stack([np.roll(x, -1, axis=0) - x, np.roll(x, -1, axis=1) - x])

    def div(p):
        return (p[0] - np.roll(p[0], 1, axis=0)) + (p[1] - np.roll(p[1], 1, axis=1))

    p = np.zeros((2,) + z.shape, np.complex128)
    for _ in range(iters):
        g = grad(div(p) - z / lam)
        n = np.sqrt(np.abs(g[0]) ** 2 + np.abs(g[1]) ** 2)
        p = (p + tau * g) / (1.0 + tau * n)
    return z - lam * div(p)


def test_tv_operators_and_prox():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((12, 10)) + 1j * rng.standard_normal((12, 10))
    q = rng.standard_normal((2, 12, 10)) + 1j * rng.standard_normal((2, 12, 10))
    assert abs(np.vdot(q, cs.tv_grad(x)) - np.vdot(cs.tv_grad_adj(q), x)) < 1e-12 * np.abs(np.vdot(q, cs.tv_grad(x)))
    v = x.copy()
    for _ in range(300):          # ||D||^2 <= 8 makes 1 / (8 lam) a valid dual step
        v = cs.tv_grad_adj(cs.tv_grad(v))
        lam_max = np.linalg.norm(v)
        v /= lam_max
    assert lam_max <= 8.0 + 1e-9
    # the dual fast gradient projection converges to the prox an independent
    # algorithm finds, and the prox minimises 1/2 |x - z|^2 + lam TV(x)
    z = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    lam = 0.3
    a = cs.tv_prox(z, lam, 3000)
    b = _chambolle_prox(z, lam)
    assert np.linalg.norm(a - b) < 1e-4 * np.linalg.norm(a)

    def obj(u):
        g = cs.tv_grad(u)
        return 0.5 * np.linalg.norm(u - z) ** 2 + lam * np.sum(np.sqrt(np.abs(g[0]) ** 2 + np.abs(g[1]) ** 2))

    f0 = obj(a)
    for _ in range(20):
        e = rng.standard_normal(z.shape) + 1j * rng.standard_normal(z.shape)
        assert obj(a + 1e-3 * e) >= f0 - 1e-9
    assert np.allclose(cs.tv_prox(np.full((8, 8), 2.0 + 1j), lam, 50), 2.0 + 1j)


def test_tv_prox_derivative_matches_differences():
    rng = np.random.default_rng(6)
    w = rng.standard_normal((2, 6, 6)) + 1j * rng.standard_normal((2, 6, 6))
    dw = rng.standard_normal((2, 6, 6)) + 1j * rng.standard_normal((2, 6, 6))
    num = (cs.ball_proj(w + 1e-7 * dw) - cs.ball_proj(w - 1e-7 * dw)) / 2e-7
    assert np.abs(cs.ball_dproj(w, dw) - num).max() < 1e-6
    z = rng.standard_normal((10, 12)) + 1j * rng.standard_normal((10, 12))
    dz = rng.standard_normal((10, 12)) + 1j * rng.standard_normal((10, 12))
    eps = 1e-8
    num = (cs.tv_prox(z + eps * dz, 0.4, 15) - cs.tv_prox(z - eps * dz, 0.4, 15)) / (2 * eps)
    d = cs.tv_dprox(z, dz, 0.4, 15)
    assert np.linalg.norm(d - num) < 1e-5 * np.linalg.norm(num)


def test_tv_fista_jvp_matches_central_differences_and_lambda_zero():
    op, b, _ = _cs_problem()
    f = cs.FistaTV(op, 2e-3, 12, inner=8)
    _, zs = f.recon(b, store=True)
    w = cs.kspace_probe(op, 4, 0)
    jw = f.jvp(w, zs)
    eps = 1e-9
    fd = (f.recon(b + eps * w) - f.recon(b - eps * w)) / (2 * eps)
    assert np.linalg.norm(jw - fd) < 1e-5 * np.linalg.norm(fd)
    f0 = cs.FistaTV(op, 0.0, 12, inner=8)
    _, zs0 = f0.recon(b, store=True)
    assert np.linalg.norm(f0.jvp(w, zs0) - f0.recon(w)) < 1e-12 * np.linalg.norm(f0.recon(w))


# ------------------------------------------------ FISTA at lam > 0 (pins)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_db4_matches_published_taps():
    h, _ = wavelet.wavelet_filter(4)
    ref = np.loadtxt(os.path.join(GOLDEN, "db4_taps.txt"))
    assert ref.shape == (8,)
    assert np.abs(h - ref).max() < 1e-13


def test_fista_momentum_weights():
    # Beck and Teboulle: t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, so
    # t_{k+1}^2 - t_{k+1} = t_k^2, t_k >= (k + 1) / 2, and the first weight
    # (t_1 - 1) / t_2 is 0 (the first step is a plain proximal-gradient step)
    op, _, f = _cs_problem(iters=40)
    t = np.array(f.t)
    assert t[0] == 1.0
    assert np.allclose(t[1:] ** 2 - t[1:], t[:-1] ** 2, rtol=1e-13)
    assert np.all(t >= (np.arange(1, t.size + 1) + 1) / 2 - 1e-12)
    assert f.theta(1) == 0.0
    for k in range(1, 41):
        assert abs(f.theta(k) - (t[k - 1] - 1.0) / t[k]) < 1e-15
    g = cs.FistaTV(op, 1e-3, 40, inner=3)
    assert g.theta(1) == 0.0 and np.allclose(g.t, f.t, rtol=0, atol=0)


def _l1_objective(op, f, b, u):
    r = op.forward(u) - b
    c = wavelet.wavedec2(u, f.levels)
    return 0.5 * np.vdot(r, r).real / f.s2 + f.lam * np.abs(c[f.mask]).sum()


def _tv_objective(op, f, b, u):
    r = op.forward(u) - b
    g = cs.tv_grad(u)
    return 0.5 * np.vdot(r, r).real / f.s2 + f.lam * np.sum(np.sqrt(np.abs(g[0]) ** 2 + np.abs(g[1]) ** 2))


def test_fista_l1_first_order_optimality():
    # minimiser of F(x) = 1/2 ||A x - b||^2 / s^2 + lam sum_detail |c_i|, c = Psi x:
    # with g = Psi A^H (b - A x) / s^2 (minus the gradient, in coefficients),
    # g = 0 on the approximation band, g = lam c / |c| on detail c != 0, and
    # |g| <= lam on detail c = 0
    op, b, f = _cs_problem(lam=2e-3, iters=1000)
    x = f.recon(b)
    g = wavelet.wavedec2(op.adjoint(b) - op.normal(x), f.levels) / f.s2
    c = wavelet.wavedec2(x, f.levels)
    a = np.abs(c)
    det = f.mask
    act = det & (a > 1e-8)
    off = det & ~act
    assert act.sum() > 100 and off.sum() > 20          # both cases occur
    assert np.abs(g[~det]).max() < 1e-6 * f.lam
    assert np.abs(g[act] - f.lam * c[act] / a[act]).max() < 1e-5 * f.lam
    assert np.abs(g[off]).max() <= f.lam * (1 + 1e-9)
    # a wrong threshold scale would move the active-set condition by that factor
    assert np.abs(g[act] - 1.05 * f.lam * c[act] / a[act]).max() > 1e-2 * f.lam


def test_fista_l1_objective_gap_bound():
    op, b, f = _cs_problem(lam=2e-3, iters=1000)
    xs = f.recon(b)
    fs = _l1_objective(op, f, b, xs)
    bound0 = 2.0 * np.vdot(xs, xs).real           # 2 L ||x_0 - x*||^2, L = 1, x_0 = 0
    for k in (1, 2, 3, 5, 10, 20, 50):
        xk = cs.FistaL1Wavelet(op, f.lam, k, levels=f.levels).recon(b)
        gap = _l1_objective(op, f, b, xk) - fs
        assert -1e-12 <= gap <= bound0 / (k + 1) ** 2


def test_fista_tv_fixed_point_of_exact_prox_gradient_map():
    # with near-exact inner solves the TV iterate is the minimiser of
    # 1/2 ||A x - b||^2 / s^2 + lam TV(x): x = prox_{lam TV}(x - grad f(x)),
    # the prox taken by the independent Chambolle solver above
    op, b, _ = _cs_problem(n=24, lam=2e-3)
    f = cs.FistaTV(op, 2e-3, 200, inner=200)
    x = f.recon(b)
    z = x - (op.normal(x) - op.adjoint(b)) / f.s2
    assert np.linalg.norm(_chambolle_prox(z, f.lam, iters=20000) - x) < 1e-6 * np.linalg.norm(x)
    # the same map with a mis-scaled prox weight is not at its fixed point
    assert np.linalg.norm(_chambolle_prox(z, 1.1 * f.lam, iters=20000) - x) > 1e-4 * np.linalg.norm(x)
    fs = _tv_objective(op, f, b, x)
    bound0 = 2.0 * np.vdot(x, x).real
    for k in (1, 2, 5, 10, 20):
        xk = cs.FistaTV(op, f.lam, k, inner=200).recon(b)
        gap = _tv_objective(op, f, b, xk) - fs
        assert -1e-9 <= gap <= bound0 / (k + 1) ** 2


def test_noise_map_jvp_estimates_diag_JJH():
    # the estimator's mean of |J w|^2 over random-phase k-space probes on the
    # sampled locations approaches diag(J J^H), J taken column by column from
    # whitened unit k-space vectors on the mask (Sec. 2.2, CS extension)
    op, b, f = _cs_problem(n=16, lam=5e-3, iters=10)
    f = cs.FistaL1Wavelet(op, 5e-3, 10, levels=1)
    _, coeffs = f.recon(b, store=True)
    exact = np.zeros((16, 16))
    idx = np.argwhere(np.broadcast_to(op.P[None] > 0, (op.nc, 16, 16)))
    for c, ky, kx in idx:
        e = np.zeros((op.nc, 16, 16), np.complex128)
        e[c, ky, kx] = 1.0
        exact += np.abs(f.jvp(e, coeffs)) ** 2
    N = 800       # Monte-Carlo error of each voxel's mean about 1 / sqrt(N) = 3.5 %
    acc = cs.noise_map_jvp(f, coeffs, 17, 0, N)
    est = acc["sum"] / acc["count"]
    rel = np.abs(est - exact) / exact
    assert acc["count"] == N
    assert np.sqrt(np.mean(rel ** 2)) < 0.08 and rel.max() < 0.35
    # a probe that also fills the unsampled locations changes nothing (A^H masks them)
    w = cs.kspace_probe(op, 3, 0)
    assert np.all(w[:, op.P == 0] == 0)
