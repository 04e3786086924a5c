/* Variable-density Poisson-disc sampling of a Cartesian k-space grid by
 * Bridson's dart throwing (Bridson, "Fast Poisson disk sampling in arbitrary
 * dimensions", SIGGRAPH 2007 sketch) with the spatially varying radius
 * r(p) = r0 (1 + 2 |p - centre| / kmax).  A candidate q is accepted when no
 * accepted point o lies closer than min(r(q), r(o)).  Random numbers come
 * from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) seeded by `seed`.
 * Input generator only; built with gcc on first use. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { uint64_t s; } rng_t;

static uint64_t splitmix64(rng_t* r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double unif(rng_t* r) { return (double)(splitmix64(r) >> 11) * 0x1p-53; }

/* Marks the sampled points in mask[ny][nx] (which the caller zeroes) and
 * returns how many points were accepted, or -1 on allocation failure. */
int poisson_disc(int ny, int nx, double r0, int k, uint64_t seed, uint8_t* mask) {
  const double cy = ny / 2.0, cx = nx / 2.0, kmax = hypot(cy, cx);
  const double cell = r0 / sqrt(2.0);
  const int gh = (int)(ny / cell) + 1, gw = (int)(nx / cell) + 1;
  const long cap = (long)gh * gw;   /* r >= r0 keeps at most one point per cell */
  int* grid = malloc(sizeof(int) * cap);
  double* py = malloc(sizeof(double) * cap);
  double* px = malloc(sizeof(double) * cap);
  double* pr = malloc(sizeof(double) * cap);
  int* active = malloc(sizeof(int) * cap);
  if (!grid || !py || !px || !pr || !active) {
    free(grid); free(py); free(px); free(pr); free(active);
    return -1;
  }
  for (long i = 0; i < cap; ++i) grid[i] = -1;
  rng_t rng = {seed};
  int n = 0, na = 0;
  py[0] = cy;
  px[0] = cx;
  pr[0] = r0;
  grid[(long)(int)(cy / cell) * gw + (int)(cx / cell)] = 0;
  n = 1;
  active[na++] = 0;
  const int reach = (int)ceil(3.0 * r0 / cell);
  while (na > 0) {
    const int ai = (int)(unif(&rng) * na);
    const int b = active[ai];
    const double rb = pr[b];
    int found = 0;
    for (int t = 0; t < k && !found; ++t) {
      const double rr = rb * (1.0 + unif(&rng));
      const double th = 2.0 * M_PI * unif(&rng);
      const double qy = py[b] + rr * sin(th), qx = px[b] + rr * cos(th);
      if (!(qy >= 0 && qy < ny && qx >= 0 && qx < nx)) continue;
      const int gy = (int)(qy / cell), gx = (int)(qx / cell);
      const double rq = r0 * (1.0 + 2.0 * hypot(qy - cy, qx - cx) / kmax);
      int ok = 1;
      const int y0 = gy - reach < 0 ? 0 : gy - reach, y1 = gy + reach + 1 > gh ? gh : gy + reach + 1;
      const int x0 = gx - reach < 0 ? 0 : gx - reach, x1 = gx + reach + 1 > gw ? gw : gx + reach + 1;
      for (int yy = y0; yy < y1 && ok; ++yy)
        for (int xx = x0; xx < x1; ++xx) {
          const int o = grid[(long)yy * gw + xx];
          if (o >= 0 && hypot(py[o] - qy, px[o] - qx) < (rq < pr[o] ? rq : pr[o])) {
            ok = 0;
            break;
          }
        }
      if (ok && grid[(long)gy * gw + gx] < 0) {
        py[n] = qy;
        px[n] = qx;
        pr[n] = rq;
        grid[(long)gy * gw + gx] = n;
        active[na++] = n;
        ++n;
        found = 1;
      }
    }
    if (!found) active[ai] = active[--na];
  }
  for (int i = 0; i < n; ++i) {
    int y = (int)py[i], x = (int)px[i];
    if (y > ny - 1) y = ny - 1;
    if (x > nx - 1) x = nx - 1;
    mask[(long)y * nx + x] = 1;
  }
  free(grid); free(py); free(px); free(pr); free(active);
  return n;
}
