// Dense per-column normal operator for phase-encode (1-D) masks on the FP32
// matrix cores.
//
// With a mask constant along kx, M is block diagonal over image columns
// (Sec. 2.1, Eq. (6) with F_x^H F_x = I): the block of column x is the
// Hermitian ny x ny matrix
//     M_x[i][j] = c(i - j) sum_c conj(S'_c[i][x]) S'_c[j][x],
//     c(d) = sum_k w_k exp(2 pi i k d / ny),  w_k = mask_k / ny,
// (S' the whitened, sign-folded maps; c the circulant F^H diag(w) F).  For K
// probes at once, q = (M_x + lam) p is a dense contraction
// [ny x ny] x [ny x K] per column, run here with v_mfma_f32_32x32x2f32.
//
// One workgroup = one column x and a tile of 32 probes; ny / 32 waves, wave w
// owning output rows [32 w, 32 w + 32).  The complex product is two real
// MFMA chains per row block (Re and Im of q), the k index of each MFMA
// carrying (Re, Im) of one p element.  The p tile sits in LDS ([ny][33]
// float2, probe fastest); the wave's slice of M_x streams from L2, read
// through the Hermitian symmetry as conj(M_x[j][i]) so that consecutive
// lanes load consecutive addresses.  The CG update of the previous iteration
// (x += alpha p, r -= alpha q, p = r + beta p) is fused in front, the four
// FP64 dot partials behind, exactly as in the FFT column kernel.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "device_common.h"
#include "runtime.h"

namespace pico {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 32;            // probes per workgroup

// G[x][j][i] = conj(M_x[i][j]), FP64 sums rounded once to FP32
__global__ void k_build_gram(const float2* __restrict__ maps, const double2* __restrict__ cvec,
                             float2* __restrict__ G, int nc, int ny) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (t >= (long)ny * ny) return;
  const int j = (int)(t / ny), i = (int)(t % ny);
  const float2* S = maps + (size_t)col * nc * ny;
  double re = 0.0, im = 0.0;   // sum_c conj(S_c[i]) S_c[j]
  for (int c = 0; c < nc; ++c) {
    const float2 a = S[(size_t)c * ny + i], b = S[(size_t)c * ny + j];
    re += (double)a.x * b.x + (double)a.y * b.y;
    im += (double)a.x * b.y - (double)a.y * b.x;
  }
  const double2 cv = cvec[((i - j) % ny + ny) % ny];
  const double mr = cv.x * re - cv.y * im, mi = cv.x * im + cv.y * re;   // M_x[i][j]
  G[((size_t)col * ny + j) * ny + i] = make_float2((float)mr, (float)-mi);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Element (row, probe) of the p / q tile: rows of 32 float2 (256 B), the
// probe index XOR-swizzled by the row so that both the column writes of the
// prologue and the row reads of the matrix loop spread over the LDS banks.
__device__ __forceinline__ int tile_at(int row, int j) { return row * kTile + (j ^ (row & 31)); }

// SMALL: ny <= 320 (at most 10 waves, an 80 KB tile): registers kept within
// six waves per SIMD so that two workgroups share a CU and one's memory
// phases overlap the other's matrix loop.
template <int MODE, bool SMALL>
__global__ __launch_bounds__(SMALL ? 640 : 1024, SMALL ? 6 : 1) void k_cart1d_gram(Cart1dArgs a,
                                                                                  const float2* __restrict__ G) {
  extern __shared__ float2 pt[];                   // [ny][32] p tile, then q tile, then reduction
  const int ny = a.ny, nw = ny / 32;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  // workgroups of one column stay on one XCD (blocks are dealt to the 8 XCDs
  // round robin), so the column's M_x is fetched into that XCD's L2 once
  const int ntiles = (a.K + kTile - 1) / kTile;
  const int b = blockIdx.x, xcd = b % 8, rest = b / 8;
  const int tile = rest % ntiles, col = xcd + 8 * (rest / ntiles);
  if (col >= a.nx) return;
  const int k0 = tile * kTile;

  // ---- prologue: wave w prepares probes j = w, w + nw, ... (column-coalesced)
  for (int j = w; j < kTile; j += nw) {
    const int k = k0 + j;
    const bool active = k < a.K;
    const size_t base = ((size_t)(active ? k : 0) * a.nx + col) * ny;
    double d0 = 0.0;
    float alpha = 0.f, beta = 0.f;
    if constexpr (MODE == C1_ITER) {
      if (active) {
        alpha = (float)a.alpha[k];
        beta = (float)a.beta[k];
      }
    }
    for (int y = lane; y < ny; y += 64) {
      float2 pv = make_float2(0.f, 0.f), rv = make_float2(0.f, 0.f);
      if (active) {
        if constexpr (MODE == C1_ITER) {
          const float2 po = a.p[base + y], qo = a.q[base + y];
          const float2 xo = a.x_zero ? make_float2(0.f, 0.f) : a.x[base + y];
          rv = cfma(a.r[base + y], -alpha, qo);
          pv = cfma(rv, beta, po);
          a.x[base + y] = cfma(xo, alpha, po);
          a.r[base + y] = rv;
          a.p[base + y] = pv;
        } else if constexpr (MODE == C1_FIRST_PROBE) {
          pv = draw_probe(a.seed, a.first + k, (uint32_t)(y * a.nx + col), 0u, a.dist);
          rv = pv;
          a.r[base + y] = pv;
          a.p[base + y] = pv;
        } else if constexpr (MODE == C1_FIRST_BUF) {
          pv = a.r[base + y];
          rv = pv;
          a.p[base + y] = pv;
        } else {   // C1_APPLY
          pv = cscale(a.src[base + y], a.scale);
        }
      }
      d0 += (double)rv.x * rv.x + (double)rv.y * rv.y;
      pt[tile_at(y, j)] = pv;
    }
    d0 = wave_sum(d0);
    if (active && lane == 0) a.part[((size_t)k * a.nx + col) * 4] = d0;
  }
  __syncthreads();

  // ---- q = M_x p on the matrix cores: rows [32 w, 32 w + 32) x 32 probes
  const int li = lane % 32, kk = lane / 32;
  const float2* __restrict__ Gc = G + (size_t)col * ny * ny + 32 * w + li;   // G[x][j][32w + li]
  floatx16 accR, accI;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    accR[v] = 0.f;
    accI[v] = 0.f;
  }
  constexpr int U = SMALL ? 4 : 8;
  float2 mA[U], mB[U];
#pragma unroll
  for (int u = 0; u < U; ++u) mA[u] = Gc[(size_t)u * ny];
  for (int c = 0; c < ny; c += 2 * U) {
#pragma unroll
    for (int u = 0; u < U; ++u) mB[u] = Gc[(size_t)(c + U + u) * ny];   // ny is a multiple of 32
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float2 m = mA[u];                           // conj(M[i][j]), j = c + u
      const float2 pp = pt[tile_at(c + u, li)];         // p[j][probe li]
      const float bv = kk ? pp.y : pp.x;
      accR = __builtin_amdgcn_mfma_f32_32x32x2f32(kk ? m.y : m.x, bv, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x2f32(kk ? m.x : -m.y, bv, accI, 0, 0, 0);
    }
    if (c + 2 * U < ny) {
#pragma unroll
      for (int u = 0; u < U; ++u) mA[u] = Gc[(size_t)(c + 2 * U + u) * ny];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float2 m = mB[u];
      const float2 pp = pt[tile_at(c + U + u, li)];
      const float bv = kk ? pp.y : pp.x;
      accR = __builtin_amdgcn_mfma_f32_32x32x2f32(kk ? m.y : m.x, bv, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f32_32x32x2f32(kk ? m.x : -m.y, bv, accI, 0, 0, 0);
    }
  }
  __syncthreads();   // every wave is done reading the p tile

  // ---- q = acc + lam p on the wave's own rows, (Re p^H q, |q|^2) partials;
  // q replaces p row by row (only this wave touches these rows now)
  double d1 = 0.0, d2 = 0.0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = 32 * w + 8 * (v / 4) + 4 * kk + (v % 4);
    const float2 p = pt[tile_at(row, li)];
    const float2 q = make_float2(fmaf(a.lam, p.x, accR[v]), fmaf(a.lam, p.y, accI[v]));
    d1 += (double)p.x * q.x + (double)p.y * q.y;
    d2 += (double)q.x * q.x + (double)q.y * q.y;
    pt[tile_at(row, li)] = q;
  }
  d1 += __shfl_xor(d1, 32, 64);   // both halves of the wave hold probe li
  d2 += __shfl_xor(d2, 32, 64);
  __syncthreads();

  // ---- epilogue: store q and the Re r^H q partial (|r|^2 went out with the prologue)
  for (int j = w; j < kTile; j += nw) {
    const int k = k0 + j;
    if (k >= a.K) continue;
    const size_t base = ((size_t)k * a.nx + col) * ny;
    double d3 = 0.0;
    for (int y = lane; y < ny; y += 64) {
      const float2 q = pt[tile_at(y, j)];
      a.q[base + y] = q;
      if constexpr (MODE != C1_APPLY) {
        const float2 r = a.r[base + y];
        d3 += (double)r.x * q.x + (double)r.y * q.y;
      }
    }
    d3 = wave_sum(d3);
    if (lane == 0) a.part[((size_t)k * a.nx + col) * 4 + 3] = d3;
  }
  __syncthreads();   // the q tile is consumed: its space takes the per-wave partials

  double* red = reinterpret_cast<double*>(pt);     // [nw][32][2]
  if (kk == 0) {
    red[(w * kTile + li) * 2] = d1;
    red[(w * kTile + li) * 2 + 1] = d2;
  }
  __syncthreads();
  if (lane < kTile && w == 0) {
    const int k = k0 + lane;
    if (k < a.K) {
      double s1 = 0.0, s2 = 0.0;
      for (int ww = 0; ww < nw; ++ww) {
        s1 += red[(ww * kTile + lane) * 2];
        s2 += red[(ww * kTile + lane) * 2 + 1];
      }
      double* pp = a.part + ((size_t)k * a.nx + col) * 4;
      pp[1] = s1;
      pp[2] = s2;
    }
  }
}

size_t gram_bytes(int ny, int nx) { return (size_t)nx * ny * ny * sizeof(float2); }

bool gram_supported(int ny) { return ny % 32 == 0 && ny >= 64 && ny <= 512; }

// c(d) = sum_k w_k exp(2 pi i k d / ny) in FP64 on the host, then the blocks
hipError_t build_gram(const float2* maps, const float* maskw_h, int nc, int ny, int nx, float2* G,
                      double2* cvec_d, hipStream_t s) {
  std::vector<double2> cv(ny);
  for (int d = 0; d < ny; ++d) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k < ny; ++k) {
      if (maskw_h[k] == 0.f) continue;
      const long ph = ((long)k * d) % ny;
      const double ang = 2.0 * M_PI * (double)ph / (double)ny;
      re += (double)maskw_h[k] * std::cos(ang);
      im += (double)maskw_h[k] * std::sin(ang);
    }
    cv[d] = make_double2(re, im);
  }
  hipError_t e = hipMemcpyAsync(cvec_d, cv.data(), ny * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)(((long)ny * ny + 255) / 256), nx), block(256);
  hipLaunchKernelGGL(k_build_gram, grid, block, 0, s, maps, cvec_d, G, nc, ny);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);   // cv leaves scope
}

template <bool SMALL>
static hipError_t launch_gram(int mode, const Cart1dArgs& a, const float2* G, hipStream_t s) {
  const int nw = a.ny / 32;
  const size_t lds = (size_t)a.ny * kTile * sizeof(float2);
  if (mode < 0 || mode > 3) return hipErrorInvalidValue;
  // allow up to 160 KiB of dynamic LDS for every mode (once per process,
  // thread-safe initialisation)
  static const hipError_t attr = [] {
    const void* fn[4] = {(const void*)k_cart1d_gram<C1_FIRST_PROBE, SMALL>, (const void*)k_cart1d_gram<C1_FIRST_BUF, SMALL>,
                         (const void*)k_cart1d_gram<C1_ITER, SMALL>, (const void*)k_cart1d_gram<C1_APPLY, SMALL>};
    for (const void* f : fn) {
      const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }();
  if (attr != hipSuccess) return attr;
  const int ntiles = (a.K + kTile - 1) / kTile;
  const int cgroups = (a.nx + 7) / 8;
  dim3 grid((unsigned)(8 * ntiles * cgroups)), block(64 * nw);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL((k_cart1d_gram<C1_FIRST_PROBE, SMALL>), grid, block, lds, s, a, G); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL((k_cart1d_gram<C1_FIRST_BUF, SMALL>), grid, block, lds, s, a, G); break;
    case C1_ITER: hipLaunchKernelGGL((k_cart1d_gram<C1_ITER, SMALL>), grid, block, lds, s, a, G); break;
    default: hipLaunchKernelGGL((k_cart1d_gram<C1_APPLY, SMALL>), grid, block, lds, s, a, G); break;
  }
  return hipGetLastError();
}

hipError_t launch_cart1d_gram(int mode, const Cart1dArgs& a, const float2* G, hipStream_t s) {
  if (!gram_supported(a.ny)) return hipErrorInvalidValue;
  if (a.ny <= 320) return launch_gram<true>(mode, a, G, s);
  return launch_gram<false>(mode, a, G, s);
}

}  // namespace pico
