// Kaiser-Bessel gridding NUFFT for non-Cartesian operators: the data path
// (A x and A^H y per coil; PMR replicas) of the spiral reconstruction
// (Sec. 3.2.2, 3.3).  The normal operator stays the exact Toeplitz form.
//
// Grid G = sigma N per axis, image placed at grid index r mod G (r centred),
// plain 2-D FFT on the grid, W x W separable Kaiser-Bessel taps per sample at
// k = floor(kappa) - W/2 + 1 + t (kappa = w G / 2 pi), de-apodisation by the
// kernel's Fourier transform at r / G, scale N^-1/2.  The adjoint is the
// exact adjoint: spread with the same weights, inverse FFT, crop.
//
// Spreading is a gather over a CSR list built once per operator (for every
// grid point, the (sample, weight) pairs whose footprint covers it, in sample
// order), so A^H is deterministic and free of atomics; interpolation gathers
// the W x W taps of each sample.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"
#include "runtime.h"

namespace pico {

// ------------------------------------------------------------------ host tables
namespace {

double bessel_i0(double x) {   // power series sum ((x/2)^2)^k / (k!)^2
  const double q = 0.25 * x * x;
  double term = 1.0, s = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * k);
    s += term;
    if (term <= 1e-17 * s) break;
  }
  return s;
}

double kb_phi(double u, int W, double beta) {
  const double a = 1.0 - (2.0 * u / W) * (2.0 * u / W);
  return a >= 0.0 ? bessel_i0(beta * std::sqrt(a)) : 0.0;
}

double kb_phi_hat(double nu, int W, double beta) {   // continuous transform of kb_phi
  const double z2 = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
  if (z2 > 1e-12) {
    const double z = std::sqrt(z2);
    return W * std::sinh(z) / z;
  }
  if (z2 < -1e-12) {
    const double z = std::sqrt(-z2);
    return W * std::sin(z) / z;
  }
  return W;
}

}  // namespace

double kb_beta(double sigma, int W) {
  return M_PI * std::sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
}

size_t KbLayout::bytes_of(size_t i) const { return sizes[i]; }

KbLayout kb_layout(long M, int W, int ny, int nx, int Gy, int Gx, int K) {
  KbLayout L;
  const size_t s[KbLayout::kParts] = {
      (size_t)M * 4,                  // ky0
      (size_t)M * 4,                  // kx0
      (size_t)M * W * 4,              // wy
      (size_t)M * W * 4,              // wx
      ((size_t)Gy * Gx + 1) * 4,      // rowptr
      (size_t)M * W * W * 4,          // entry sample
      (size_t)M * W * W * 4,          // entry weight
      (size_t)ny * 4,                 // dy
      (size_t)nx * 4,                 // dx
      (size_t)Gx * 8,                 // twiddles x
      (size_t)Gy * 8,                 // twiddles y
      (size_t)K * Gy * Gx * 8,        // grid [K][Gy][Gx]
      (size_t)K * M * 8,              // samples [K][M]
  };
  for (int i = 0; i < KbLayout::kParts; ++i) L.sizes[i] = s[i];
  return L;
}

// Fill the tables (host double precision, stored float32).  traj_h: [M][2].
void kb_build_host(const float* traj_h, long M, int W, double sigma, int ny, int nx, int Gy, int Gx,
                   std::vector<int>& ky0, std::vector<int>& kx0, std::vector<float>& wy,
                   std::vector<float>& wx, std::vector<int>& rowptr, std::vector<int>& ent_m,
                   std::vector<float>& ent_w, std::vector<float>& dy, std::vector<float>& dx) {
  const double beta = kb_beta(sigma, W);
  ky0.resize(M);
  kx0.resize(M);
  wy.resize((size_t)M * W);
  wx.resize((size_t)M * W);
  auto taps = [&](double w, int G, int& k0m, float* wt) {
    const double kappa = w * G / (2.0 * M_PI);
    const long k0 = (long)std::floor(kappa) - W / 2 + 1;
    for (int t = 0; t < W; ++t) wt[t] = (float)kb_phi(kappa - (double)(k0 + t), W, beta);
    k0m = (int)(((k0 % G) + G) % G);
  };
  for (long m = 0; m < M; ++m) {
    taps((double)traj_h[2 * m], Gy, ky0[m], &wy[(size_t)m * W]);
    taps((double)traj_h[2 * m + 1], Gx, kx0[m], &wx[(size_t)m * W]);
  }
  // CSR over grid points, entries in (sample, ty, tx) order within a row
  const size_t G2 = (size_t)Gy * Gx;
  rowptr.assign(G2 + 1, 0);
  for (long m = 0; m < M; ++m)
    for (int a = 0; a < W; ++a)
      for (int b = 0; b < W; ++b) {
        const int iy = (ky0[m] + a) % Gy, ix = (kx0[m] + b) % Gx;
        ++rowptr[(size_t)iy * Gx + ix + 1];
      }
  for (size_t g = 0; g < G2; ++g) rowptr[g + 1] += rowptr[g];
  ent_m.resize((size_t)M * W * W);
  ent_w.resize((size_t)M * W * W);
  std::vector<int> fill(rowptr.begin(), rowptr.end() - 1);
  for (long m = 0; m < M; ++m)
    for (int a = 0; a < W; ++a)
      for (int b = 0; b < W; ++b) {
        const int iy = (ky0[m] + a) % Gy, ix = (kx0[m] + b) % Gx;
        const int pos = fill[(size_t)iy * Gx + ix]++;
        ent_m[pos] = (int)m;
        ent_w[pos] = wy[(size_t)m * W + a] * wx[(size_t)m * W + b];
      }
  dy.resize(ny);
  dx.resize(nx);
  for (int y = 0; y < ny; ++y) dy[y] = (float)(1.0 / kb_phi_hat((double)(y - ny / 2) / Gy, W, beta));
  for (int x = 0; x < nx; ++x) dx[x] = (float)(1.0 / kb_phi_hat((double)(x - nx / 2) / Gx, W, beta));
}

// ------------------------------------------------------------------ kernels

// nbuf[b][m] = CN(0, 1) Philox draw (stream 1, element c M + m, draw first + b)
__global__ void k_kb_noise(float2* __restrict__ nbuf, int M, int c, uint64_t seed, uint64_t first) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (m >= M) return;
  nbuf[(size_t)b * M + m] = draw_probe(seed, first + b, (uint32_t)((size_t)c * M + m), 1u, 3);
}

// grid[b][g] = sum over the CSR row g of w * src[b * bstride + m]
__global__ void k_kb_spread(const float2* __restrict__ src, long bstride, const int* __restrict__ rowptr,
                            const int* __restrict__ ent_m, const float* __restrict__ ent_w,
                            float2* __restrict__ grid, long G2) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (g >= G2) return;
  const float2* sb = src + (size_t)b * bstride;
  float2 acc = make_float2(0.f, 0.f);
  for (int e = rowptr[g], e1 = rowptr[g + 1]; e < e1; ++e) acc = cfma(acc, ent_w[e], sb[ent_m[e]]);
  grid[(size_t)b * G2 + g] = acc;
}

// out[b][y][x] (= or +=) conj(S_c[y][x]) grid[b][(y - ny/2) mod Gy][(x - nx/2) mod Gx] dy dx scale
__global__ void k_kb_crop_combine(const float2* __restrict__ grid, const float2* __restrict__ Sc,
                                  const float* __restrict__ dy, const float* __restrict__ dx,
                                  float2* __restrict__ out, int ny, int nx, int Gy, int Gx, float scale,
                                  int accumulate) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= (long)ny * nx) return;
  const int y = (int)(i / nx), x = (int)(i % nx);
  const int gy = (y - ny / 2 + Gy) % Gy, gx = (x - nx / 2 + Gx) % Gx;
  const float2 v = cscale(grid[(size_t)b * Gy * Gx + (size_t)gy * Gx + gx], dy[y] * dx[x] * scale);
  const float2 t = cmulc(Sc[i], v);
  float2* o = out + (size_t)b * ny * nx + i;
  *o = accumulate ? cadd(*o, t) : t;
}

// grid[b] = S_c x[b] dy dx scale placed at (r mod G), zero elsewhere
__global__ void k_kb_expand(const float2* __restrict__ xin, const float2* __restrict__ Sc,
                            const float* __restrict__ dy, const float* __restrict__ dx,
                            float2* __restrict__ grid, int ny, int nx, int Gy, int Gx, float scale) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (g >= (long)Gy * Gx) return;
  const int gy = (int)(g / Gx), gx = (int)(g % Gx);
  const int ry = gy < ny / 2 ? gy : (gy >= Gy - ny / 2 ? gy - Gy : Gy);   // Gy: outside
  const int rx = gx < nx / 2 ? gx : (gx >= Gx - nx / 2 ? gx - Gx : Gx);
  float2 v = make_float2(0.f, 0.f);
  if (ry != Gy && rx != Gx) {
    const int y = ry + ny / 2, x = rx + nx / 2;
    const size_t i = (size_t)y * nx + x;
    v = cscale(cmul(Sc[i], xin[(size_t)b * ny * nx + i]), dy[y] * dx[x] * scale);
  }
  grid[(size_t)b * Gy * Gx + g] = v;
}

// out[b * bstride + m] = sum_{a, t} wy[m][a] wx[m][t] grid[b][ky0 + a][kx0 + t]
__global__ void k_kb_interp(const float2* __restrict__ grid, const int* __restrict__ ky0,
                            const int* __restrict__ kx0, const float* __restrict__ wy,
                            const float* __restrict__ wx, float2* __restrict__ out, long bstride, int M,
                            int W, int Gy, int Gx) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (m >= M) return;
  const float2* gb = grid + (size_t)b * Gy * Gx;
  float2 acc = make_float2(0.f, 0.f);
  int iy = ky0[m];
  for (int a = 0; a < W; ++a, ++iy) {
    if (iy >= Gy) iy -= Gy;
    const float wa = wy[(size_t)m * W + a];
    int ix = kx0[m];
    for (int t = 0; t < W; ++t, ++ix) {
      if (ix >= Gx) ix -= Gx;
      acc = cfma(acc, wa * wx[(size_t)m * W + t], gb[(size_t)iy * Gx + ix]);
    }
  }
  out[(size_t)b * bstride + m] = acc;
}

static dim3 kb_grid(long n, int K) { return dim3((unsigned)((n + 255) / 256), K); }

// out[K][ny][nx] = A^H of K multi-coil sample arrays: src [K][nc][M] (whitened),
// or Philox CN(0, 1) noise (src == nullptr; stream 1, element c M + m)
hipError_t kb_adjoint(const KbOp& o, const float2* maps, int nc, int K, const float2* src, uint64_t seed,
                      uint64_t first, float2* out, hipStream_t s) {
  const long G2 = (long)o.Gy * o.Gx, n = (long)o.ny * o.nx;
  const float scale = (float)(1.0 / std::sqrt((double)n));
  for (int c = 0; c < nc; ++c) {
    const float2* sp;
    long bstride;
    if (src) {
      sp = src + (size_t)c * o.M;
      bstride = (long)nc * o.M;
    } else {
      hipLaunchKernelGGL(k_kb_noise, kb_grid(o.M, K), dim3(256), 0, s, o.samples, (int)o.M, c, seed, first);
      sp = o.samples;
      bstride = o.M;
    }
    hipLaunchKernelGGL(k_kb_spread, kb_grid(G2, K), dim3(256), 0, s, sp, bstride, o.rowptr, o.ent_m,
                       o.ent_w, o.grid, G2);
    hipError_t e = launch_fft2d(o.grid, K, o.Gy, o.Gx, true, o.twx, o.twy, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kb_crop_combine, kb_grid(n, K), dim3(256), 0, s, o.grid, maps + (size_t)c * n,
                       o.dy, o.dx, out, o.ny, o.nx, o.Gy, o.Gx, scale, c > 0 ? 1 : 0);
  }
  return hipGetLastError();
}

// out[K][nc][M] = A x for K images x [K][ny][nx]
hipError_t kb_forward(const KbOp& o, const float2* maps, int nc, int K, const float2* x, float2* out,
                      hipStream_t s) {
  const long G2 = (long)o.Gy * o.Gx, n = (long)o.ny * o.nx;
  const float scale = (float)(1.0 / std::sqrt((double)n));
  for (int c = 0; c < nc; ++c) {
    hipLaunchKernelGGL(k_kb_expand, kb_grid(G2, K), dim3(256), 0, s, x, maps + (size_t)c * n, o.dy, o.dx,
                       o.grid, o.ny, o.nx, o.Gy, o.Gx, scale);
    hipError_t e = launch_fft2d(o.grid, K, o.Gy, o.Gx, false, o.twx, o.twy, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kb_interp, kb_grid(o.M, K), dim3(256), 0, s, o.grid, o.ky0, o.kx0, o.wy, o.wx,
                       out + (size_t)c * o.M, (long)nc * o.M, (int)o.M, o.W, o.Gy, o.Gx);
  }
  return hipGetLastError();
}

}  // namespace pico
