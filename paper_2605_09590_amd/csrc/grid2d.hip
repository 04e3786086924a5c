// Normal operator on a 2-D frequency grid, shared by Cartesian 2-D masks and
// the non-Cartesian Toeplitz embedding:
//
//   q = lam p + sum_c conj(S_c) . crop( G2^-1( W . G2( pad(S_c . p) ) ) )
//
// where G2 is the unnormalised 2-D DFT on a Gy x Gx grid and W a real
// weight, transposed [Gx][Gy] in memory:
//  * Cartesian 2-D mask: Gy x Gx = ny x nx, W = mask / (ny nx), maps folded
//    with (-1)^(y+x) (the centred DFT is (-1)^((ny+nx)/2) D F D, D = (-1)^(y+x),
//    so the centred-order mask applies unchanged; Sec. 2.1 Eq. (6));
//  * spiral, Toeplitz form (Sec. 3.2.2, 3.3): Gy x Gx = 2ny x 2nx,
//    W = DFT(circulant embedding of the point-spread function) / (4 ny nx),
//    real because the PSF is Hermitian; the product is the exact NUDFT
//    normal operator A^H A.
//
// Three kernels per application, all per-probe fields row-major [K][ny][nx]:
//  rows_fwd  per image row: CG update / probe draw, then per coil S_c p,
//            zero-pad to Gx, row FFT -> T[k][c][y][Gx] (only the ny
//            non-zero rows of the padded grid are stored);
//  cols      per tile of adjacent grid columns of one (k, c) plane, staged
//            through LDS for coalescing: zero-pad to Gy, column FFT,
//            times W, inverse column FFT, keep rows < ny;
//  rows_inv  per image row: per coil inverse row FFT, crop to nx,
//            conj(S_c) times it, summed over coils; q written with the FP64
//            partial dots of the CG step.
#include "fft.h"
#include "runtime.h"

namespace pico {

template <int L>
__device__ __forceinline__ double group_reduce2(double v, double* red, int lane) {
  red[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (lane == 0) {
    for (int i = 0; i < L; ++i) s += red[threadIdx.x + i];
  }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- row pass 1
template <class CF, int MODE>
__global__ __launch_bounds__(64) void k_rows_fwd(Grid2dArgs a) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ double red[64];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const long gid = (long)blockIdx.x * G + g;
  const bool active = g < G && gid < (long)a.K * a.ny;
  const long gg = active ? gid : 0;
  const int k = (int)(gg / a.ny), y = (int)(gg % a.ny);
  const bool inA = CF::inA(lane), inB = CF::inB(lane);
  float2* lds = lds_all + g * CF::SPAN;
  typename CF::Tw tw;
  CF::load_tw(tw, a.twx, lane);

  const size_t rowoff = ((size_t)k * a.ny + y) * a.nx;
  // the per-probe fields never alias one another: restrict lets every load of
  // the row go out before the first store
  float2* __restrict__ X = a.x;
  float2* __restrict__ R = a.r;
  float2* __restrict__ P = a.p;
  const float2* __restrict__ Q = a.q;
  const float2* __restrict__ SRC = a.src;
  float2 pv[CF::VMAX];
  double d0 = 0.0;
  float alpha = 0.f, beta = 0.f;
  if constexpr (MODE == C1_ITER) {
    alpha = (float)a.alpha[k];
    beta = (float)a.beta[k];
  }
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    const int xx = CF::posA(lane, m);
    const bool ok = inA && xx < a.nx;
    const size_t i = rowoff + (ok ? xx : 0);   // in-bounds address for every lane
    float2 val = make_float2(0.f, 0.f);
    if constexpr (MODE == C1_FIRST_PROBE) {
      val = draw_probe(a.seed, a.first + k, (uint32_t)(y * a.nx + xx), 0u, a.dist);
      if (!ok) val = make_float2(0.f, 0.f);
      if (active && ok) { R[i] = val; P[i] = val; }
      d0 += (double)val.x * val.x + (double)val.y * val.y;
    } else if constexpr (MODE == C1_FIRST_BUF) {
      val = ok ? R[i] : make_float2(0.f, 0.f);
      if (active && ok) P[i] = val;
      d0 += (double)val.x * val.x + (double)val.y * val.y;
    } else if constexpr (MODE == C1_ITER) {
      val = make_float2(0.f, 0.f);   // the update runs below, all loads first
    } else {  // C1_APPLY
      val = ok ? cscale(SRC[i], a.scale) : make_float2(0.f, 0.f);
    }
    pv[m] = val;
  }
  if constexpr (MODE == C1_ITER) {
    // finish iteration i-1 and start i: x += alpha p, r -= alpha q, p = r + beta p.
    // In chunks of H elements, every load of a chunk is issued before its first store.
    constexpr int H = VA > 8 ? 8 : VA;
    const bool xz = a.x_zero != 0;
#pragma unroll
    for (int m0 = 0; m0 < VA; m0 += H) {
      float2 po[H], qo[H], ro[H], xo[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (m0 + h >= VA) break;
        const int xx = CF::posA(lane, m0 + h);
        const size_t i = rowoff + ((inA && xx < a.nx) ? xx : 0);
        po[h] = P[i];
        qo[h] = Q[i];
        ro[h] = R[i];
        xo[h] = X[i];
      }
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int m = m0 + h;
        if (m >= VA) break;
        const int xx = CF::posA(lane, m);
        const bool ok = inA && xx < a.nx;
        const size_t i = rowoff + (ok ? xx : 0);
        const float2 rn = ok ? cfma(ro[h], -alpha, qo[h]) : make_float2(0.f, 0.f);
        pv[m] = ok ? cfma(rn, beta, po[h]) : make_float2(0.f, 0.f);
        if (active && ok) {
          X[i] = cfma(xz ? make_float2(0.f, 0.f) : xo[h], alpha, po[h]);
          R[i] = rn;
          P[i] = pv[m];
        }
        d0 += (double)rn.x * rn.x + (double)rn.y * rn.y;
      }
    }
  }
  if constexpr (MODE != C1_APPLY) {
    d0 = group_reduce2<L>(d0, red, lane);
    if (active && lane == 0) a.part[((size_t)k * a.ny + y) * 4] = d0;
  }

  float2* __restrict__ T = a.T;
  uint32_t* __restrict__ Tb = a.Tb;
  for (int c = 0; c < a.nc; ++c) {
    const MapRef s = MapRef{a.maps, a.maps_bf} + ((size_t)c * a.ny + y) * a.nx;
    float2 v[CF::VMAX];
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      const int xx = CF::posA(lane, m);
      const bool ok = inA && xx < a.nx;
      const float2 sv = s[ok ? xx : 0];
      v[m] = ok ? cmul(sv, pv[m]) : make_float2(0.f, 0.f);
    }
    CF::template forward<false>(v, lds, lane, tw);
    if (active && inB) {
      const size_t off = (((size_t)k * a.nc + c) * a.ny + y) * a.Gx;
      if (Tb) {
#pragma unroll
        for (int r = 0; r < VB; ++r) Tb[off + CF::posB(lane, r)] = pack_bf16x2(v[r]);
      } else {
#pragma unroll
        for (int r = 0; r < VB; ++r) T[off + CF::posB(lane, r)] = v[r];
      }
    }
  }
}

// ---------------------------------------------------------------- column strips
// Strip of `ncol` (<= ngrp) adjacent columns of one plane to / from an LDS tile
// [rows][ts].  Loads go out in batches of 8 per thread before any is consumed,
// so a workgroup keeps 8 x 256 loads in flight instead of one per thread.
__device__ __forceinline__ float2 widen(float2 v) { return v; }
__device__ __forceinline__ float2 widen(uint32_t v) { return unpack_bf16x2(v); }
__device__ __forceinline__ void narrow(float2& d, float2 v) { d = v; }
__device__ __forceinline__ void narrow(uint32_t& d, float2 v) { d = pack_bf16x2(v); }

// E: float2 (complex64 planes) or uint32_t (packed bfloat16 pairs)
template <class E>
__device__ __forceinline__ void strip_load(float2* __restrict__ tile, const E* __restrict__ src,
                                           int rows, int ngrp, int ts, int ncol, long stride) {
  constexpr int B = 8;
  const int total = rows * ngrp;
  for (int i0 = threadIdx.x; i0 < total; i0 += B * 256) {
    E v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = i0 + u * 256;
      const int yy = i / ngrp, j = i % ngrp;
      v[u] = (i < total && j < ncol) ? src[(size_t)yy * stride + j] : E{};
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = i0 + u * 256;
      if (i < total) tile[(i / ngrp) * ts + i % ngrp] = widen(v[u]);
    }
  }
}

template <class E>
__device__ __forceinline__ void strip_store(const float2* __restrict__ tile, E* __restrict__ dst,
                                            int rows, int ngrp, int ts, int ncol, long stride) {
  const int total = rows * ngrp;
  for (int i = threadIdx.x; i < total; i += 256) {
    const int yy = i / ngrp, j = i % ngrp;
    if (j < ncol) narrow(dst[(size_t)yy * stride + j], tile[yy * ts + j]);
  }
}

// ---------------------------------------------------------------- column pass
// One workgroup of 256 lanes: NGRP = 256 / L column groups, one grid column
// each, adjacent columns of one (k, c) plane.
template <class CF>
__global__ __launch_bounds__(256) void k_cols(Grid2dArgs a) {
  constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  constexpr int TS = NGRP + 1;  // padded tile row
  extern __shared__ float2 dyn[];
  float2* tile = dyn;                                  // [ny][TS]
  float2* xch = dyn + (size_t)a.ny * TS;               // NG exchange regions
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int x0 = blockIdx.x * NGRP;
  const size_t plane = (size_t)blockIdx.y * a.ny * a.Gx;
  const int ncol = min(NGRP, a.Gx - x0);
  if (a.Tb) strip_load(tile, a.Tb + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
  else strip_load(tile, a.T + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
  __syncthreads();
  const bool grp = g < NGRP && g < ncol;
  const bool inA = CF::inA(lane), inB = CF::inB(lane);
  typename CF::Tw tw;
  CF::load_tw(tw, a.twy, lane);
  float2 v[CF::VMAX];
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    const int yy = CF::posA(lane, m);
    v[m] = (grp && inA && yy < a.ny) ? tile[yy * TS + g] : make_float2(0.f, 0.f);
  }
  float2* lds = xch + g * CF::SPAN;
  CF::template forward<false>(v, lds, lane, tw);
  const float* __restrict__ wcol = a.w + (size_t)(grp ? x0 + g : 0) * a.Gy;
  if (inB) {
#pragma unroll
    for (int r = 0; r < VB; ++r) v[r] = cscale(v[r], wcol[CF::posB(lane, r)]);
  }
  CF::template inverse<true>(v, lds, lane, tw);
  if (grp && inA) {
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      const int yy = CF::posA(lane, m);
      if (yy < a.ny) tile[yy * TS + g] = v[m];
    }
  }
  __syncthreads();
  if (a.Tb) strip_store(tile, a.Tb + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
  else strip_store(tile, a.T + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
}

// ---------------------------------------------------------------- row pass 2
template <class CF, int MODE>
__global__ __launch_bounds__(64) void k_rows_inv(Grid2dArgs a) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ double red[64];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const long gid = (long)blockIdx.x * G + g;
  const bool active = g < G && gid < (long)a.K * a.ny;
  const long gg = active ? gid : 0;
  const int k = (int)(gg / a.ny), y = (int)(gg % a.ny);
  const bool inA = CF::inA(lane), inB = CF::inB(lane);
  float2* lds = lds_all + g * CF::SPAN;
  typename CF::Tw tw;
  CF::load_tw(tw, a.twx, lane);
  const size_t rowoff = ((size_t)k * a.ny + y) * a.nx;

  const float2* __restrict__ P = a.p;
  const float2* __restrict__ R = a.r;
  const float2* __restrict__ SRC = a.src;
  const float2* __restrict__ T = a.T;
  float2* __restrict__ Qo = a.q;
  // p (or scale * src) of this row: lam p enters q first (when lam != 0); the
  // dots at the end load it again
  auto load_p = [&](float2* pa) {
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      const int xx = CF::posA(lane, m);
      const bool ok = inA && xx < a.nx;
      const size_t i = rowoff + (ok ? xx : 0);
      const float2 pval = MODE == C1_APPLY ? cscale(SRC[i], a.scale) : P[i];
      pa[m] = ok ? pval : make_float2(0.f, 0.f);
    }
  };
  float2 qa[CF::VMAX];
  if (a.lam != 0.f) {
    load_p(qa);
#pragma unroll
    for (int m = 0; m < VA; ++m) qa[m] = cscale(qa[m], a.lam);
  } else {
#pragma unroll
    for (int m = 0; m < VA; ++m) qa[m] = make_float2(0.f, 0.f);
  }
  for (int c = 0; c < a.nc; ++c) {
    float2 v[CF::VMAX];
    const size_t off = (((size_t)k * a.nc + c) * a.ny + y) * a.Gx;
    if (a.Tb) {
#pragma unroll
      for (int r = 0; r < VB; ++r) v[r] = inB ? unpack_bf16x2(a.Tb[off + CF::posB(lane, r)]) : make_float2(0.f, 0.f);
    } else {
#pragma unroll
      for (int r = 0; r < VB; ++r) v[r] = inB ? T[off + CF::posB(lane, r)] : make_float2(0.f, 0.f);
    }
    CF::template inverse<true>(v, lds, lane, tw);
    const MapRef s = MapRef{a.maps, a.maps_bf} + ((size_t)c * a.ny + y) * a.nx;
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      const int xx = CF::posA(lane, m);
      const bool ok = inA && xx < a.nx;
      const float2 sv = s[ok ? xx : 0];
      if (ok) qa[m] = cadd(qa[m], cmulc(sv, v[m]));
    }
  }
  float2 pa[CF::VMAX], ra[CF::VMAX];
  load_p(pa);
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    const int xx = CF::posA(lane, m);
    const size_t i = rowoff + ((inA && xx < a.nx) ? xx : 0);
    ra[m] = MODE == C1_ITER ? R[i] : pa[m];
  }
  double d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    const int xx = CF::posA(lane, m);
    const bool ok = inA && xx < a.nx;
    const size_t i = rowoff + (ok ? xx : 0);
    const float2 rv = ra[m];
    if (ok) {
      if (active) Qo[i] = qa[m];
      d1 += (double)pa[m].x * qa[m].x + (double)pa[m].y * qa[m].y;
      d2 += (double)qa[m].x * qa[m].x + (double)qa[m].y * qa[m].y;
      d3 += (double)rv.x * qa[m].x + (double)rv.y * qa[m].y;
    }
  }
  d1 = group_reduce2<L>(d1, red, lane);
  d2 = group_reduce2<L>(d2, red, lane);
  d3 = group_reduce2<L>(d3, red, lane);
  if (active && lane == 0) {
    double* pp = a.part + ((size_t)k * a.ny + y) * 4;
    pp[1] = d1;
    pp[2] = d2;
    pp[3] = d3;
  }
}

// ---------------------------------------------------------------- plans
using L64 = TwoStep<8, 8>;
using L96 = StockhamCol<FFTPlan<96, 8, 12, 4, 2>>;
using L128 = StockhamCol<FFTPlan<128, 16, 8, 4, 4>>;
using L160 = StockhamCol<FFTPlan<160, 8, 20, 4, 2>>;
using L192 = StockhamCol<FFTPlan<192, 16, 12, 4, 4>>;
using L256 = TwoStep<16, 16>;
using L288 = StockhamCol<FFTPlan<288, 16, 18, 2, 2, 2, 2>>;
using L320 = TwoStep<20, 16>;
using L384 = StockhamCol<FFTPlan<384, 16, 24, 4, 4>>;
using L512 = StockhamCol<FFTPlan<512, 32, 16, 16, 2>>;
using L576 = StockhamCol<FFTPlan<576, 16, 36, 4, 4>>;
using L640 = StockhamCol<FFTPlan<640, 32, 20, 4, 4, 2>>;
using L768 = StockhamCol<FFTPlan<768, 32, 24, 4, 4, 2>>;

bool grid_line_supported(int n) {
  switch (n) {
    case 64: case 96: case 128: case 160: case 192: case 256: case 288: case 320: case 384:
    case 512: case 576: case 640: case 768:
      return true;
    default:
      return false;
  }
}

template <class F>
static hipError_t with_line(int n, F&& f) {
  switch (n) {
    case 64: return f(L64{});
    case 96: return f(L96{});
    case 128: return f(L128{});
    case 160: return f(L160{});
    case 192: return f(L192{});
    case 256: return f(L256{});
    case 288: return f(L288{});
    case 320: return f(L320{});
    case 384: return f(L384{});
    case 512: return f(L512{});
    case 576: return f(L576{});
    case 640: return f(L640{});
    case 768: return f(L768{});
    default: return hipErrorInvalidValue;
  }
}

template <class CF>
static hipError_t rows_fwd(int mode, const Grid2dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  const long rows = (long)a.K * a.ny;
  dim3 grid((unsigned)((rows + G - 1) / G)), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL((k_rows_fwd<CF, C1_FIRST_PROBE>), grid, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL((k_rows_fwd<CF, C1_FIRST_BUF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_rows_fwd<CF, C1_ITER>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_rows_fwd<CF, C1_APPLY>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class CF>
static hipError_t rows_inv(int mode, const Grid2dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  const long rows = (long)a.K * a.ny;
  dim3 grid((unsigned)((rows + G - 1) / G)), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: case C1_FIRST_BUF:
      hipLaunchKernelGGL((k_rows_inv<CF, C1_FIRST_BUF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_rows_inv<CF, C1_ITER>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_rows_inv<CF, C1_APPLY>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class CF>
static hipError_t cols(const Grid2dArgs& a, hipStream_t s) {
  constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
  const size_t lds = ((size_t)a.ny * (NGRP + 1) + (size_t)NG * CF::SPAN) * sizeof(float2);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static bool attr_set = false;   // allow more than the default 64 KiB of dynamic LDS
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cols<CF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  dim3 grid((a.Gx + NGRP - 1) / NGRP, (unsigned)((long)a.K * a.nc)), block(256);
  hipLaunchKernelGGL((k_cols<CF>), grid, block, lds, s, a);
  return hipGetLastError();
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
  hipError_t e = with_line(a.Gx, [&](auto cf) { return rows_fwd<decltype(cf)>(mode, a, s); });
  if (e != hipSuccess) return e;
  e = with_line(a.Gy, [&](auto cf) { return cols<decltype(cf)>(a, s); });
  if (e != hipSuccess) return e;
  return with_line(a.Gx, [&](auto cf) { return rows_inv<decltype(cf)>(mode, a, s); });
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
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fft_cols<CF, INV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
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
                            int ny, int nx, uint64_t seed, uint64_t first, uint32_t stream, int dist,
                            float scale) {
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
        v = draw_probe(seed, first + b, (uint32_t)((size_t)c * n + i), stream, dist);
      }
    }
    out[((size_t)b * nc + c) * n + i] = cscale(v, sg);
  }
}

hipError_t launch_kspace_in(const float2* src, const double* linv, const uint8_t* mask, float2* out,
                            int B, int nc, int ny, int nx, uint64_t seed, uint64_t first,
                            uint32_t stream, int dist, float scale, hipStream_t s) {
  const long n = (long)ny * nx;
  dim3 grid((unsigned)((n + 255) / 256), B), block(256);
  hipLaunchKernelGGL(k_kspace_in, grid, block, 0, s, src, linv, mask, out, B, nc, ny, nx, seed,
                     first, stream, dist, scale);
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
      const float2 v = draw_probe(a.seed, a.first + k, (uint32_t)i, 0u, a.dist);
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

__global__ void k_quantise_maps(float2* __restrict__ maps, uint32_t* __restrict__ bf, long count) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t w = pack_bf16x2(maps[i]);
  bf[i] = w;
  maps[i] = unpack_bf16x2(w);
}

hipError_t launch_quantise_maps(float2* maps, uint32_t* bf, long count, hipStream_t s) {
  hipLaunchKernelGGL(k_quantise_maps, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, maps, bf, count);
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
