// Reduced-resolution noise grid (Sec. 5, Discussion: the noise map follows
// the smooth coil geometry, so it can be estimated on a coarser grid and
// interpolated back).  The coarse problem of factor f is the acquisition
// restricted to the central (ny/f) x (nx/f) block of k-space on an
// (ny/f) x (nx/f) grid; with the centred orthonormal DFT coarse pixel m sits
// at native pixel f m, so the coarse maps are the native maps at every f-th
// pixel, and the variance level carries over without rescaling.
#include "device_common.h"
#include "runtime.h"

namespace pico {

namespace {

// out[c][my][mx] = maps[c][f my][f mx]
__global__ void k_subsample_maps(const float2* __restrict__ maps, float2* __restrict__ out, int nc, int ny,
                                 int nx, int f) {
  const int cy = ny / f, cx = nx / f;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nc * cy * cx) return;
  const int mx = (int)(i % cx);
  const long t = i / cx;
  const int my = (int)(t % cy), c = (int)(t / cy);
  out[i] = maps[((size_t)c * ny + (size_t)f * my) * nx + (size_t)f * mx];
}

// native pixel (y, x) at coarse coordinate (y / f, x / f): periodic bilinear
__global__ void k_upsample_bilinear(const double* __restrict__ coarse, double* __restrict__ out, int cy, int cx,
                                    int f) {
  const int ny = cy * f, nx = cx * f;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)ny * nx) return;
  const int y = (int)(i / nx), x = (int)(i % nx);
  const int y0 = y / f, x0 = x / f;
  const int y1 = y0 + 1 < cy ? y0 + 1 : 0, x1 = x0 + 1 < cx ? x0 + 1 : 0;
  const double wy = (double)(y - y0 * f) / f, wx = (double)(x - x0 * f) / f;
  const double a = coarse[(long)y0 * cx + x0], b = coarse[(long)y0 * cx + x1];
  const double c = coarse[(long)y1 * cx + x0], d = coarse[(long)y1 * cx + x1];
  out[i] = (1.0 - wy) * ((1.0 - wx) * a + wx * b) + wy * ((1.0 - wx) * c + wx * d);
}

}  // namespace

hipError_t launch_subsample_maps(const float2* maps, float2* out, int nc, int ny, int nx, int f, hipStream_t s) {
  const long total = (long)nc * (ny / f) * (nx / f);
  hipLaunchKernelGGL(k_subsample_maps, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, maps, out, nc, ny,
                     nx, f);
  return hipGetLastError();
}

hipError_t launch_upsample_bilinear(const double* coarse, double* out, int cy, int cx, int f, hipStream_t s) {
  const long total = (long)cy * f * cx * f;
  hipLaunchKernelGGL(k_upsample_bilinear, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, coarse, out, cy,
                     cx, f);
  return hipGetLastError();
}

}  // namespace pico
