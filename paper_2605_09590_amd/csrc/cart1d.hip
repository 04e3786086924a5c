// Separable Cartesian SENSE: launch of the normal operator (kernels in
// cart1d_normal.h; cart1d_bf16.hip holds the bfloat16-map instantiation) and
// the CG building blocks of the column-major layout.
#include "cart1d_normal.h"

namespace pico {

bool cart1d_supported(int ny) {
  switch (ny) {
    case 64: case 96: case 128: case 160: case 192: case 256: case 288: case 320: case 384: case 512:
      return true;
    default:
      return false;
  }
}

hipError_t launch_cart1d(int mode, const Cart1dArgs& a, hipStream_t s) {
  if (a.maps_bf) return launch_cart1d_bf16(mode, a, s);
  return cart1d_dispatch<false>(mode, a, s);
}

// ------------------------------------------------------------ map preparation
// out[col][c][y] = (-1)^y sum_d Linv[c][d] maps[d][y][col]  (whitening, Sec. 2.1 Eq. (3))
__global__ void k_prep_maps_cart1d(const float2* __restrict__ maps, const double* __restrict__ linv,
                                   float2* __restrict__ out, int nc, int ny, int nx) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (y >= ny) return;
  const double sg = (y & 1) ? -1.0 : 1.0;
  for (int c = 0; c < nc; ++c) {
    double re = 0.0, im = 0.0;
    for (int d = 0; d <= c; ++d) {
      const double lr = linv[2 * (c * nc + d)], li = linv[2 * (c * nc + d) + 1];
      const float2 m = maps[((size_t)d * ny + y) * nx + col];
      re += lr * m.x - li * m.y;
      im += lr * m.y + li * m.x;
    }
    out[((size_t)col * nc + c) * ny + y] = make_float2((float)(sg * re), (float)(sg * im));
  }
}

hipError_t launch_prep_maps_cart1d(const float2* maps, const double* linv, float2* out, int nc,
                                   int ny, int nx, hipStream_t s) {
  dim3 grid((ny + 63) / 64, nx), block(64);
  hipLaunchKernelGGL(k_prep_maps_cart1d, grid, block, 0, s, maps, linv, out, nc, ny, nx);
  return hipGetLastError();
}

// ------------------------------------------------------------ power-method start
__global__ void k_power_start(float2* __restrict__ p, int ny, int nx) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (y >= ny) return;
  const float s = rsqrtf((float)ny * (float)nx);
  const float2 v = draw_probe(0, 0, (uint32_t)(y * nx + col), 3u, 0);
  p[(size_t)col * ny + y] = cscale(v, s);
}

hipError_t launch_power_start(float2* p, int ny, int nx, hipStream_t s) {
  dim3 grid((ny + 63) / 64, nx), block(64);
  hipLaunchKernelGGL(k_power_start, grid, block, 0, s, p, ny, nx);
  return hipGetLastError();
}

// ------------------------------------------------------------ exact diagonal by row probing
// For a phase-encode mask Sigma is block diagonal over image columns, so the
// probe that is 1 on image row y0 + k of every column returns column x's
// Sigma_x e_(y0+k): its entry on that row is diag(Sigma) there.
__global__ void k_unit_rows(float2* __restrict__ r, int y0, int ny, int nx) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y, k = blockIdx.z;
  if (y >= ny) return;
  r[((size_t)k * nx + col) * ny + y] = make_float2(y == y0 + k ? 1.f : 0.f, 0.f);
}

__global__ void k_extract_rows(const float2* __restrict__ x, double* __restrict__ var, int K, int y0,
                               int ny, int nx) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (col >= nx || k >= K) return;
  const int y = y0 + k;
  var[(size_t)y * nx + col] = (double)x[((size_t)k * nx + col) * ny + y].x;
}

hipError_t launch_unit_rows(float2* r, int K, int y0, int ny, int nx, hipStream_t s) {
  dim3 grid((ny + 63) / 64, nx, K), block(64);
  hipLaunchKernelGGL(k_unit_rows, grid, block, 0, s, r, y0, ny, nx);
  return hipGetLastError();
}

hipError_t launch_extract_rows(const float2* x, double* var, int K, int y0, int ny, int nx,
                               hipStream_t s) {
  dim3 grid((nx + 63) / 64, K), block(64);
  hipLaunchKernelGGL(k_extract_rows, grid, block, 0, s, x, var, K, y0, ny, nx);
  return hipGetLastError();
}

// ------------------------------------------------------------ accumulation
// PICO: sum += Re(conj v x), sum_im += Im(conj v x), sumsq += Re(.)^2 over the
// K probes of the tile, in probe order (App. A, Algorithm 1).  PMR: sum +=
// x, sumsq += |x|^2.
__global__ void k_accum_colmajor(AccumArgs a) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (y >= a.ny) return;
  const uint32_t vox = (uint32_t)(y * a.nx + col);
  double s = 0.0, si = 0.0, ss = 0.0;
  for (int k = 0; k < a.K; ++k) {
    const float2 u = a.x[((size_t)k * a.nx + col) * a.ny + y];
    if (a.pmr) {
      s += (double)u.x;
      si += (double)u.y;
      ss += (double)u.x * u.x + (double)u.y * u.y;
    } else {
      const float2 v = draw_probe(arg_seed(a), arg_first(a) + k, vox, 0u, a.dist);
      const double re = (double)v.x * u.x + (double)v.y * u.y;
      const double im = (double)v.x * u.y - (double)v.y * u.x;
      s += re;
      si += im;
      ss += re * re;
    }
  }
  a.sum[vox] += s;
  if (a.sum_im) a.sum_im[vox] += si;
  if (a.sumsq) a.sumsq[vox] += ss;
}

hipError_t launch_accum_colmajor(const AccumArgs& a, hipStream_t s) {
  dim3 grid((a.ny + 63) / 64, a.nx), block(64);
  hipLaunchKernelGGL(k_accum_colmajor, grid, block, 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ layout changes
// v [K][ny][nx] (row-major images) -> out [K][nx][ny]
__global__ void k_transpose_in(const float2* __restrict__ v, float2* __restrict__ out, int ny, int nx) {
  __shared__ float2 tile[32][33];
  const int k = blockIdx.z;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const float2* vk = v + (size_t)k * ny * nx;
  float2* ok = out + (size_t)k * ny * nx;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int y = y0 + i, x = x0 + threadIdx.x;
    if (y < ny && x < nx) tile[i][threadIdx.x] = vk[(size_t)y * nx + x];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int x = x0 + i, y = y0 + threadIdx.x;
    if (y < ny && x < nx) ok[(size_t)x * ny + y] = tile[threadIdx.x][i];
  }
}

// x [K][nx][ny] -> u [K][ny][nx]
__global__ void k_transpose_out(const float2* __restrict__ x, float2* __restrict__ u, int ny, int nx) {
  __shared__ float2 tile[32][33];
  const int k = blockIdx.z;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const float2* xk = x + (size_t)k * ny * nx;
  float2* uk = u + (size_t)k * ny * nx;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int x = x0 + i, y = y0 + threadIdx.x;
    if (y < ny && x < nx) tile[i][threadIdx.x] = xk[(size_t)x * ny + y];
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int y = y0 + i, xx = x0 + threadIdx.x;
    if (y < ny && xx < nx) uk[(size_t)y * nx + xx] = tile[threadIdx.x][i];
  }
}

hipError_t launch_transpose_in(const float2* v, float2* out, int K, int ny, int nx, hipStream_t s) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, K), block(32, 8);
  hipLaunchKernelGGL(k_transpose_in, grid, block, 0, s, v, out, ny, nx);
  return hipGetLastError();
}

hipError_t launch_transpose_out(const float2* x, float2* u, int K, int ny, int nx, hipStream_t s) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, K), block(32, 8);
  hipLaunchKernelGGL(k_transpose_out, grid, block, 0, s, x, u, ny, nx);
  return hipGetLastError();
}

}  // namespace pico
