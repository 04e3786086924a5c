"""The seeded input generators: determinism and the stated structure of the
variable-density Poisson-disc masks (spacing rule, acceleration, calibration)."""
import math

import numpy as np

import workloads


def test_poisson_disc_mask_properties():
    ny, nx, R, calib = 96, 128, 2.0, 12
    m = workloads.poisson_disc_mask(ny, nx, R, calib, seed=4)
    assert m.dtype == np.uint8 and m.shape == (ny, nx)
    assert abs(m.size / m.sum() - R) <= 0.01 * R
    c = m[ny // 2 - calib // 2: ny // 2 + calib // 2, nx // 2 - calib // 2: nx // 2 + calib // 2]
    assert c.all()
    assert np.array_equal(m, workloads.poisson_disc_mask(ny, nx, R, calib, seed=4))
    assert not np.array_equal(m, workloads.poisson_disc_mask(ny, nx, R, calib, seed=5))
    # density falls with |k|: the centre band is denser than the periphery
    yy, xx = np.meshgrid(np.arange(ny) - ny / 2, np.arange(nx) - nx / 2, indexing="ij")
    rad = np.hypot(yy, xx) / math.hypot(ny / 2, nx / 2)
    inner = m[(rad < 0.3) & ~((abs(yy) < calib / 2) & (abs(xx) < calib / 2))].mean()
    outer = m[rad > 0.7].mean()
    assert inner > 1.5 * outer


def test_poisson_disc_spacing_rule():
    # the raw sampler (no calibration block): every pair of points is at least
    # min(r(a), r(b)) apart, with r(p) = r0 (1 + 2 |p - c| / kmax); the points
    # are marked on the grid, so compare after flooring (slack of one cell diagonal)
    ny, nx, r0 = 64, 64, 1.3
    m = workloads._poisson_disc(ny, nx, r0, 0, seed=9)
    pts = np.argwhere(m > 0).astype(float)
    cy, cx = ny / 2, nx / 2
    kmax = math.hypot(cy, cx)
    r = r0 * (1 + 2 * np.hypot(pts[:, 0] - cy, pts[:, 1] - cx) / kmax)
    d = np.hypot(pts[:, None, 0] - pts[None, :, 0], pts[:, None, 1] - pts[None, :, 1])
    lim = np.minimum(r[:, None], r[None, :]) - math.sqrt(2) - 2 * r0 / kmax * math.sqrt(2)
    np.fill_diagonal(d, np.inf)
    assert (d >= lim).all()
    assert len(pts) > 200
