"""Pins of the oracle's Philox and probe distributions.

The round structure is pinned against numpy's library Philox4x64-10 (same
published construction, 64-bit constants); the probe families against the
moment conditions of Sec. 2.2, Eq. (15), and the kurtosis values of App. B.
"""
import numpy as np
import pytest

from oracle import philox


def test_philox4x64_matches_numpy_library():
    key = np.array([0x0123456789ABCDEF, 0x0FEDCBA987654321], np.uint64)
    for start in (0, 5, 2**40 + 3):
        bg = np.random.Philox(key=key, counter=np.array([start, 7, 0, 1], np.uint64))
        raw = [int(x) for x in bg.random_raw(8)]
        # numpy increments the 256-bit counter before each block
        mine = (philox.philox_scalar([start + 1, 7, 0, 1], key.tolist(), bits=64)
                + philox.philox_scalar([start + 2, 7, 0, 1], key.tolist(), bits=64))
        assert raw == list(mine)


def test_vectorised_matches_scalar_4x32():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, size=(4, 50), dtype=np.uint64)
    k0, k1 = 0xDEADBEEF, 0x12345678
    vec = philox.philox4x32(*ctr, k0, k1)
    for j in range(50):
        ref = philox.philox_scalar(ctr[:, j].tolist(), [k0, k1], bits=32)
        assert tuple(int(v[j]) for v in vec) == ref


def test_phase_fraction_uniform_and_moments():
    n = 1 << 18
    w0, _, _, _ = philox.draw_words(11, 0, n, philox.STREAM_PROBE)
    f = philox.phase_fraction(w0)
    hist = np.bincount((f * 64).astype(int), minlength=64)
    chi2 = ((hist - n / 64) ** 2 / (n / 64)).sum()
    assert chi2 < 63 + 6 * np.sqrt(2 * 63)          # ~6 sigma
    v = np.exp(2j * np.pi * f)
    assert abs(v.mean()) < 6 / np.sqrt(n)
    assert abs((v * v).mean()) < 6 / np.sqrt(n)      # circular: E[v^2] = 0


@pytest.mark.parametrize("dist,kappa", [("phase", 1.0), ("qpsk", 1.0),
                                        ("rademacher", 1.0), ("gaussian", 2.0)])
def test_probe_families_moments(dist, kappa):
    n = 1 << 17
    v = philox.probe(5, 3, n, dist)
    assert abs(v.mean()) < 6 / np.sqrt(n)
    assert abs(np.mean(np.abs(v) ** 2) - 1) < 6 * np.sqrt(kappa) / np.sqrt(n) + 1e-12
    assert abs(np.mean(np.abs(v) ** 4) - kappa) < 0.05


def test_draws_independent_across_probe_index_and_stream():
    a = philox.probe(1, 0, 4096)
    b = philox.probe(1, 1, 4096)
    c = philox.probe(1, 0, 4096, stream=philox.STREAM_PMR)
    for x, y in ((a, b), (a, c)):
        assert abs(np.vdot(x, y)) / 4096 < 6 / np.sqrt(4096)
