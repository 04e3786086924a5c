// Normal operator on a 2-D frequency grid (complex64 storage), the batched
// 2-D FFT and the elementwise kernels of the grid path.  The operator's
// kernels are in grid2d_normal.h; grid2d_bf16.hip instantiates them for
// bfloat16 storage.
#include "grid2d_normal.h"

namespace pico {

bool grid_line_supported(int n) {
  switch (n) {
    case 64: case 96: case 128: case 160: case 192: case 256: case 288: case 320: case 384:
    case 512: case 576: case 640: case 768:
      return true;
    default:
      return false;
  }
}

size_t grid_cols_lds_bytes(int Gy, int ny) {
  size_t out = 0;
  (void)with_line(Gy, [&](auto cf) {
    using CF = decltype(cf);
    constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
    out = ((size_t)ny * (NGRP + 1) + (size_t)NG * CF::SPAN) * sizeof(float2);
    return hipSuccess;
  });
  return out;
}

hipError_t launch_grid_normal(int mode, const Grid2dArgs& a, hipStream_t s) {
  if (a.maps_bf) return launch_grid_normal_bf16(mode, a, s);
  return grid_normal<0>(mode, a, s);
}

// ---------------------------------------------------------------- standalone batched 2-D FFT
// In-place unnormalised transform of B planes [B][ny][nx] (rows, then columns).
template <class CF, bool INV>
__global__ __launch_bounds__(64) void k_fft_lines(float2* data, long nlines, const float2* twt) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  __shared__ float2 lds_all[NG * CF::SPAN];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const long line = (long)blockIdx.x * G + g;
  const bool active = g < G && line < nlines;
  float2* d = data + (size_t)(active ? line : 0) * CF::N;
  typename CF::Tw tw;
  CF::load_tw(tw, twt, lane);
  float2 v[CF::VMAX];
#pragma unroll
  for (int m = 0; m < CF::VA; ++m) v[m] = CF::inA(lane) ? d[CF::posA(lane, m)] : make_float2(0.f, 0.f);
  CF::template forward<INV>(v, lds_all + g * CF::SPAN, lane, tw);
  if (active && CF::inB(lane)) {
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) d[CF::posB(lane, r)] = v[r];
  }
}

template <class CF, bool INV>
__global__ __launch_bounds__(256) void k_fft_cols(float2* data, int ny, int nx, const float2* twt) {
  constexpr int L = CF::L, NGRP = 256 / L;
  constexpr int TS = NGRP + 1;
  extern __shared__ float2 dyn[];
  float2* tile = dyn;
  float2* xch = dyn + (size_t)ny * TS;
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int x0 = blockIdx.x * NGRP;
  const size_t plane = (size_t)blockIdx.y * ny * nx;
  const int ncol = min(NGRP, nx - x0);
  strip_load(tile, data + plane + x0, ny, NGRP, TS, ncol, nx);
  __syncthreads();
  const bool grp = g < NGRP && g < ncol;
  typename CF::Tw tw;
  CF::load_tw(tw, twt, lane);
  float2 v[CF::VMAX];
#pragma unroll
  for (int m = 0; m < CF::VA; ++m)
    v[m] = (grp && CF::inA(lane)) ? tile[CF::posA(lane, m) * TS + g] : make_float2(0.f, 0.f);
  CF::template forward<INV>(v, xch + g * CF::SPAN, lane, tw);
  __syncthreads();   // every group has read its column before rows are overwritten
  if (grp && CF::inB(lane)) {
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) tile[CF::posB(lane, r) * TS + g] = v[r];
  }
  __syncthreads();
  strip_store(tile, data + plane + x0, ny, NGRP, TS, ncol, nx);
}

template <class CF, bool INV>
static hipError_t fft_cols(float2* data, long planes, int ny, int nx, const float2* twt, hipStream_t s) {
  constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
  const size_t lds = ((size_t)ny * (NGRP + 1) + (size_t)NG * CF::SPAN) * sizeof(float2);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // allow more than the default 64 KiB of dynamic LDS (once per process,
  // thread-safe initialisation)
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_fft_cols<CF, INV>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  dim3 grid((nx + NGRP - 1) / NGRP, (unsigned)planes), block(256);
  hipLaunchKernelGGL((k_fft_cols<CF, INV>), grid, block, lds, s, data, ny, nx, twt);
  return hipGetLastError();
}

hipError_t launch_fft2d(float2* data, long planes, int ny, int nx, bool inverse, const float2* twx,
                        const float2* twy, hipStream_t s) {
  const long nlines = planes * ny;
  hipError_t e = with_line(nx, [&](auto cf) {
    using CF = decltype(cf);
    constexpr int G = 64 / CF::L;
    dim3 grid((unsigned)((nlines + G - 1) / G)), block(64);
    if (inverse) hipLaunchKernelGGL((k_fft_lines<CF, true>), grid, block, 0, s, data, nlines, twx);
    else hipLaunchKernelGGL((k_fft_lines<CF, false>), grid, block, 0, s, data, nlines, twx);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return with_line(ny, [&](auto cf) {
    using CF = decltype(cf);
    return inverse ? fft_cols<CF, true>(data, planes, ny, nx, twy, s)
                   : fft_cols<CF, false>(data, planes, ny, nx, twy, s);
  });
}

// ---------------------------------------------------------------- gridding normal operator: image-row passes
// The coil image (ny x nx, centred) sits on the oversampled grid (Gy x Gx)
// at rows (y - ny/2) mod Gy and columns (x - nx/2) mod Gx; every other point
// of the expanded image is zero, and only those rows and columns are read
// back after the inverse transform.  So the row transforms run on the ny
// image rows only, kept compactly ([K][ny][Gx], row y), and the column
// transforms read (forward) or write (inverse) just those rows of the grid.

// image index of grid index g (line of G points, image of n), -1 outside
__device__ __forceinline__ int crop_index(int g, int n, int G) {
  return g < n / 2 ? g + n / 2 : (g >= G - n / 2 ? g - (G - n / 2) : -1);
}

// forward: out[b][y] = FFT_Gx of the grid row of image row y, which holds
// S_c x[b] dy dx scale at columns (x - nx/2) mod Gx.  inverse: the inverse
// FFT_Gx of in[b][y] cropped to the image, de-apodised, times conj(S_c) and
// written (or added, accumulate) to out[b][y][x].  One row per group of L
// lanes; every load goes out from an in-bounds address.
template <class CF, bool INV>
__global__ __launch_bounds__(64) void k_kbn_rows(const float2* __restrict__ in, const float2* __restrict__ Sc,
                                                 const float* __restrict__ dy, const float* __restrict__ dx,
                                                 float2* __restrict__ out, long nlines, int ny, int nx, float scale,
                                                 int accumulate, const float2* __restrict__ twx) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  __shared__ float2 lds_all[NG * CF::SPAN];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const long line = (long)blockIdx.x * G + g;
  const bool active = g < G && line < nlines;
  const long ln = active ? line : 0;
  const int y = (int)(ln % ny);
  typename CF::Tw tw;
  CF::load_tw(tw, twx, lane);
  const float fy = dy[y] * scale;
  const float2* sr = Sc + (size_t)y * nx;
  float2 v[CF::VMAX];
  if constexpr (!INV) {
    const float2* xr = in + (size_t)ln * nx;   // image row y of probe ln / ny
#pragma unroll
    for (int m = 0; m < CF::VA; ++m) {
      const int x = CF::inA(lane) ? crop_index(CF::posA(lane, m), nx, CF::N) : -1;
      const int xs = x >= 0 ? x : 0;
      v[m] = cscale(cmul(sr[xs], xr[xs]), x >= 0 ? fy * dx[xs] : 0.f);
    }
  } else {
    const float2* ir = in + (size_t)ln * CF::N;
#pragma unroll
    for (int m = 0; m < CF::VA; ++m) {
      const bool ok = CF::inA(lane);
      v[m] = cscale(ir[ok ? CF::posA(lane, m) : 0], ok ? 1.f : 0.f);
    }
  }
  CF::template forward<INV>(v, lds_all + g * CF::SPAN, lane, tw);
  if (!active || !CF::inB(lane)) return;
  if constexpr (!INV) {
    float2* o = out + (size_t)ln * CF::N;
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) o[CF::posB(lane, r)] = v[r];
  } else {
    float2* o = out + (size_t)ln * nx;
    float2 prev[CF::VMAX];
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) {
      const int x = crop_index(CF::posB(lane, r), nx, CF::N);
      prev[r] = accumulate ? o[x >= 0 ? x : 0] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) {
      const int x = crop_index(CF::posB(lane, r), nx, CF::N);
      const int xs = x >= 0 ? x : 0;
      const float2 t = cmulc(sr[xs], cscale(v[r], fy * dx[xs]));
      if (x >= 0) o[x] = cadd(prev[r], t);
    }
  }
}

// Column transforms of B planes between the compact image rows and the full
// grid: forward reads in[b] = [ny][Gx] (image row y is grid row (y - ny/2)
// mod Gy, zero elsewhere) and writes out[b] = [Gy][Gx]; inverse reads all Gy
// rows of in[b] and writes only the image rows, out[b] = [ny][Gx].  The strip
// tile doubles as the groups' exchange regions once every group holds its
// column in registers.
template <class CF, bool INV>
__global__ __launch_bounds__(256) void k_fft_cols_crop(const float2* __restrict__ in, float2* __restrict__ out,
                                                       int ny, int Gx, const float2* __restrict__ twt) {
  constexpr int L = CF::L, NGRP = 256 / L, TS = NGRP + 1, GY = CF::N;
  extern __shared__ float2 dyn[];
  float2* tile = dyn;
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int x0 = blockIdx.x * NGRP;
  const size_t b = blockIdx.y;
  const int ncol = min(NGRP, Gx - x0);
  const int rows_in = INV ? GY : ny, rows_out = INV ? ny : GY;
  strip_load(tile, in + b * rows_in * Gx + x0, rows_in, NGRP, TS, ncol, Gx);
  __syncthreads();
  const bool grp = g < NGRP && g < ncol;
  typename CF::Tw tw;
  CF::load_tw(tw, twt, lane);
  float2 v[CF::VMAX];
#pragma unroll
  for (int m = 0; m < CF::VA; ++m) {
    const int gy = CF::posA(lane, m);
    const int row = INV ? gy : crop_index(gy, ny, GY);
    v[m] = (grp && CF::inA(lane) && row >= 0) ? tile[row * TS + g] : make_float2(0.f, 0.f);
  }
  __syncthreads();   // every group holds its column: the tile becomes the exchange regions
  CF::template forward<INV>(v, dyn + g * CF::SPAN, lane, tw);
  __syncthreads();   // every transform is done before outputs overwrite the exchange regions
  if (grp && CF::inB(lane)) {
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) {
      const int gy = CF::posB(lane, r);
      const int row = INV ? crop_index(gy, ny, GY) : gy;
      if (row >= 0) tile[row * TS + g] = v[r];
    }
  }
  __syncthreads();
  strip_store(tile, out + b * rows_out * Gx + x0, rows_out, NGRP, TS, ncol, Gx);
}

hipError_t launch_kbn_rows(bool inverse, const float2* in, const float2* Sc, const float* dy, const float* dx,
                           float2* out, int K, int ny, int nx, int Gx, float scale, int accumulate,
                           const float2* twx, hipStream_t s) {
  const long nlines = (long)K * ny;
  return with_line(Gx, [&](auto cf) {
    using CF = decltype(cf);
    constexpr int G = 64 / CF::L;
    const dim3 grid((unsigned)((nlines + G - 1) / G)), block(64);
    if (inverse)
      hipLaunchKernelGGL((k_kbn_rows<CF, true>), grid, block, 0, s, in, Sc, dy, dx, out, nlines, ny, nx, scale,
                         accumulate, twx);
    else
      hipLaunchKernelGGL((k_kbn_rows<CF, false>), grid, block, 0, s, in, Sc, dy, dx, out, nlines, ny, nx, scale,
                         accumulate, twx);
    return hipGetLastError();
  });
}

template <class CF, bool INV>
static hipError_t cols_crop(const float2* in, float2* out, long planes, int ny, int Gx, const float2* twy,
                            hipStream_t s) {
  constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
  const size_t lds = std::max((size_t)CF::N * (NGRP + 1), (size_t)NG * CF::SPAN) * sizeof(float2);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_fft_cols_crop<CF, INV>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((Gx + NGRP - 1) / NGRP), (unsigned)planes), block(256);
  hipLaunchKernelGGL((k_fft_cols_crop<CF, INV>), grid, block, lds, s, in, out, ny, Gx, twy);
  return hipGetLastError();
}

hipError_t launch_fft_cols_crop(const float2* in, float2* out, long planes, int ny, int Gy, int Gx, bool inverse,
                                const float2* twy, hipStream_t s) {
  return with_line(Gy, [&](auto cf) {
    using CF = decltype(cf);
    return inverse ? cols_crop<CF, true>(in, out, planes, ny, Gx, twy, s)
                   : cols_crop<CF, false>(in, out, planes, ny, Gx, twy, s);
  });
}

// ---------------------------------------------------------------- k-space inputs
// out[b][c][ky][kx] = f(b, c, ky, kx) * mask[ky][kx] * (-1)^(ky+kx) * scale, where f
// is the measured data whitened here (src and linv given, b = 0:
// sum_d Linv[c][d] src[d]), caller k-space arrays already whitened (src only,
// [B][nc][ny][nx]), or a Philox draw (counter element (c ny + ky) nx + kx, draw first + b, given stream and
// family).  With scale = (-1)^((ny+nx)/2) / sqrt(ny nx), an unnormalised inverse
// 2-D FFT and a combine with conj(S') give A^H of the k-space array, since the
// centred orthonormal DFT is (-1)^((ny+nx)/2) D F D / sqrt(ny nx).
__global__ void k_kspace_in(const float2* __restrict__ src, const double* __restrict__ linv,
                            const uint8_t* __restrict__ mask, float2* __restrict__ out, int B, int nc,
                            int ny, int nx, uint64_t seed, uint64_t first, const uint64_t* __restrict__ tp,
                            uint32_t stream, int dist, float scale) {
  const long n = (long)ny * nx;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n || b >= B) return;
  const int ky = (int)(i / nx), kx = (int)(i % nx);
  const float sg = ((ky + kx) & 1) ? -scale : scale;
  for (int c = 0; c < nc; ++c) {
    float2 v = make_float2(0.f, 0.f);
    if (mask[i]) {
      if (src && !linv) {
        v = src[((size_t)b * nc + c) * n + i];   // already whitened, per-b arrays
      } else if (src) {
        double re = 0.0, im = 0.0;
        for (int d = 0; d <= c; ++d) {
          const double lr = linv[2 * (c * nc + d)], li = linv[2 * (c * nc + d) + 1];
          const float2 m = src[(size_t)d * n + i];
          re += lr * m.x - li * m.y;
          im += lr * m.y + li * m.x;
        }
        v = make_float2((float)re, (float)im);
      } else {
        v = tp ? draw_probe(tp[0], tp[1] + b, (uint32_t)((size_t)c * n + i), stream, dist)
               : draw_probe(seed, first + b, (uint32_t)((size_t)c * n + i), stream, dist);
      }
    }
    out[((size_t)b * nc + c) * n + i] = cscale(v, sg);
  }
}

hipError_t launch_kspace_in(const float2* src, const double* linv, const uint8_t* mask, float2* out,
                            int B, int nc, int ny, int nx, uint64_t seed, uint64_t first,
                            const uint64_t* tp, uint32_t stream, int dist, float scale, hipStream_t s) {
  const long n = (long)ny * nx;
  dim3 grid((unsigned)((n + 255) / 256), B), block(256);
  hipLaunchKernelGGL(k_kspace_in, grid, block, 0, s, src, linv, mask, out, B, nc, ny, nx, seed,
                     first, tp, stream, dist, scale);
  return hipGetLastError();
}

// out[b][i] = sum_c conj(S'_c[i]) T[b][c][i]
__global__ void k_coil_combine(const float2* __restrict__ T, const float2* __restrict__ maps,
                               float2* __restrict__ out, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  float2 acc = make_float2(0.f, 0.f);
  for (int c = 0; c < nc; ++c) acc = cadd(acc, cmulc(maps[(size_t)c * n + i], T[((size_t)b * nc + c) * n + i]));
  out[(size_t)b * n + i] = acc;
}

hipError_t launch_coil_combine(const float2* T, const float2* maps, float2* out, int B, int nc,
                               long n, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), B), block(256);
  hipLaunchKernelGGL(k_coil_combine, grid, block, 0, s, T, maps, out, nc, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- row-major accumulation
__global__ void k_accum_rowmajor(AccumArgs a) {
  const int n = a.ny * a.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, si = 0.0, ss = 0.0;
  for (int k = 0; k < a.K; ++k) {
    const float2 u = a.x[(size_t)k * n + i];
    if (a.pmr) {
      s += (double)u.x;
      si += (double)u.y;
      ss += (double)u.x * u.x + (double)u.y * u.y;
    } else {
      const float2 v = draw_probe(arg_seed(a), arg_first(a) + k, (uint32_t)i, 0u, a.dist);
      const double re = (double)v.x * u.x + (double)v.y * u.y;
      const double im = (double)v.x * u.y - (double)v.y * u.x;
      s += re;
      si += im;
      ss += re * re;
    }
  }
  a.sum[i] += s;
  if (a.sum_im) a.sum_im[i] += si;
  if (a.sumsq) a.sumsq[i] += ss;
}

hipError_t launch_accum_rowmajor(const AccumArgs& a, hipStream_t s) {
  const int n = a.ny * a.nx;
  hipLaunchKernelGGL(k_accum_rowmajor, dim3((n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- map preparation
// out[c][y][x] = sg(y, x) sum_d Linv[c][d] maps[d][y][x]; sg = (-1)^(y+x) when fold.
__global__ void k_prep_maps_rowmajor(const float2* __restrict__ maps, const double* __restrict__ linv,
                                     float2* __restrict__ out, int nc, int ny, int nx, int fold) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ny * nx) return;
  const int y = i / nx, x = i % nx;
  const double sg = (fold && ((y + x) & 1)) ? -1.0 : 1.0;
  for (int c = 0; c < nc; ++c) {
    double re = 0.0, im = 0.0;
    for (int d = 0; d <= c; ++d) {
      const double lr = linv[2 * (c * nc + d)], li = linv[2 * (c * nc + d) + 1];
      const float2 m = maps[(size_t)d * ny * nx + i];
      re += lr * m.x - li * m.y;
      im += lr * m.y + li * m.x;
    }
    out[(size_t)c * ny * nx + i] = make_float2((float)(sg * re), (float)(sg * im));
  }
}

hipError_t launch_prep_maps_rowmajor(const float2* maps, const double* linv, float2* out, int nc,
                                     int ny, int nx, int fold, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_maps_rowmajor, dim3((ny * nx + 255) / 256), dim3(256), 0, s, maps, linv,
                     out, nc, ny, nx, fold);
  return hipGetLastError();
}

// w[kx][ky] = mask[ky][kx] * scale (Cartesian 2-D weights, transposed)
__global__ void k_mask_weights(const uint8_t* __restrict__ mask, float* __restrict__ w, int ny, int nx,
                               float scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ny * nx) return;
  const int ky = i / nx, kx = i % nx;
  w[(size_t)kx * ny + ky] = mask[i] ? scale : 0.f;
}

__global__ void k_quantise_maps(float2* __restrict__ maps, uint32_t* __restrict__ bf, long count, int round_copy) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t w = pack_bf16x2(maps[i]);
  bf[i] = w;
  if (round_copy) maps[i] = unpack_bf16x2(w);
}

hipError_t launch_quantise_maps(float2* maps, uint32_t* bf, long count, bool round_copy, hipStream_t s) {
  hipLaunchKernelGGL(k_quantise_maps, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, maps, bf, count,
                     round_copy ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_mask_weights(const uint8_t* mask, float* w, int ny, int nx, float scale,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_mask_weights, dim3((ny * nx + 255) / 256), dim3(256), 0, s, mask, w, ny, nx,
                     scale);
  return hipGetLastError();
}

__global__ void k_power_start_rowmajor(float2* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = cscale(draw_probe(0, 0, (uint32_t)i, 3u, 0), rsqrtf((float)n));
}

hipError_t launch_power_start_rowmajor(float2* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_power_start_rowmajor, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace pico
