// Kernels of the normal operator on a 2-D frequency grid, shared by Cartesian
// 2-D masks and the non-Cartesian Toeplitz embedding (templates; each storage
// kind is instantiated in a translation unit of its own):
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
#pragma once

#include <algorithm>
#include <type_traits>

#include "fft.h"
#include "runtime.h"

namespace pico {
// Coil map value i as stored (complex64, or for ST >= 1 a packed bfloat16
// pair) and widened; prefetched values stay in storage form until use, so
// the loads are not waited on at the point of issue
template <int ST> using MapElem = std::conditional_t<(ST >= 1), uint32_t, float2>;
template <int ST>
__device__ __forceinline__ MapElem<ST> map_raw(const Grid2dArgs& a, size_t i) {
  if constexpr (ST >= 1) return a.maps_bf[i];
  else return a.maps[i];
}
__device__ __forceinline__ float2 widen(float2 v) { return v; }
__device__ __forceinline__ float2 widen(uint32_t v) { return unpack_bf16x2(v); }
template <int ST>
__device__ __forceinline__ float2 map_at(const Grid2dArgs& a, size_t i) { return widen(map_raw<ST>(a, i)); }


// Direct global -> LDS copy of one row of n elements of E per column group of
// the wavefront: group gi's row, from src(gi), goes to the start of its
// transform tile.  Each lane loads 16 bytes per instruction and the hardware
// places them at tile + lane * 16 bytes, so the loads hold no registers.
// The row kernels use it to fetch the next coil's row into the tile, which is
// idle between two transforms; wait_lds_loads() precedes the first LDS read
// of the row.  Rows are 16-byte aligned (n and the row pitch multiples of
// 16 / E).
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima): the direct
// LDS loads count as vector memory operations, and their data is in LDS once
// the counter has drained.  Issued explicitly before the first read of a
// fetched row: the compiler does not order LDS reads after these loads.
__device__ __forceinline__ void wait_lds_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <class CF, class E, int GS, class F>
__device__ __forceinline__ void dma_rows(E* dst, int n, F&& src) {
  constexpr int G = 64 / CF::L, PER = 16 / (int)sizeof(E), CH = 64 * PER;
  const int lo = (int)threadIdx.x * PER;   // this lane's first element of every chunk
#pragma unroll
  for (int gi = 0; gi < G; ++gi) {
    const E* s = src(gi) + lo;
    E* d = dst + gi * GS;
#pragma unroll
    for (int j = 0; j * CH < CF::N; ++j)   // rows are at most N elements
      if (j * CH + lo < n)
        __builtin_amdgcn_global_load_lds((const void*)(s + j * CH),
                                         (__attribute__((address_space(3))) void*)(d + j * CH), 16, 0, 0);
  }
}

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
template <class CF, int MODE, int ST, bool HALF>
__global__ __launch_bounds__(64) void k_rows_fwd(Grid2dArgs a) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  // HALF (the Toeplitz grids, nx = Gx / 2): values m >= VA / 2 lie past the
  // image row, so they are compile-time zeros in the forward transform
  constexpr int VAH = HALF ? VA / 2 : VA;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ double red[64 + L];   // lane 0 of a partial last group reads L entries
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const long gid = (long)blockIdx.x * G + g;
  const bool active = g < G && gid < (long)a.K * a.ny;
  const long gg = active ? gid : 0;
  const int k = (int)(gg / a.ny), y = (int)(gg % a.ny);
  const bool inA = CF::inA(lane), inB = CF::inB(lane);
  float2* lds = lds_all + g * CF::SPAN;
  typename CF::Tw tw;
  CF::load_tw(tw, a.twx, lane);
  // two-step rows (256 points and more): coil 0's map rows go into the
  // transform tiles while the CG update runs (later coils': see the coil loop)
  constexpr bool DMA = CF::kRowsDma, PF = !DMA && CF::N >= 384;
  using ME = MapElem<ST>;
  auto map_rows = [&](int c) {
    dma_rows<CF, ME, CF::SPAN * (int)(sizeof(float2) / sizeof(ME))>(reinterpret_cast<ME*>(lds_all), a.nx, [&](int gi) {
      const long gq = (long)blockIdx.x * G + gi;
      const long gr = gq < (long)a.K * a.ny ? gq : 0;
      const size_t moff = ((size_t)c * a.ny + (int)(gr % a.ny)) * a.nx;
      if constexpr (ST >= 1) return (const ME*)(a.maps_bf + moff);
      else return (const ME*)(a.maps + moff);
    });
  };
  if constexpr (DMA) map_rows(0);

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
    if (HALF && m >= VAH) {   // past the image row
      pv[m] = make_float2(0.f, 0.f);
      continue;
    }
    const int xx = CF::posA(lane, m);
    const bool ok = inA && xx < a.nx;
    const size_t i = rowoff + (ok ? xx : 0);   // in-bounds address for every lane
    float2 val = make_float2(0.f, 0.f);
    if constexpr (MODE == C1_FIRST_PROBE) {
      val = draw_probe(arg_seed(a), arg_first(a) + k, (uint32_t)(y * a.nx + xx), 0u, a.dist);
      if (!ok) val = make_float2(0.f, 0.f);
      if (active && ok) { R[i] = val; P[i] = val; }
      d0 += (double)val.x * val.x + (double)val.y * val.y;
    } else if constexpr (MODE == C1_FIRST_BUF) {
      // loads go out on every lane (the address is in bounds) and lanes
      // outside the row are zeroed by a factor: a load under a lane
      // condition (or as an operand of a select) gets a branch and a wait
      // of its own
      val = cscale(R[i], ok ? 1.f : 0.f);
      if (active && ok) P[i] = val;
      d0 += (double)val.x * val.x + (double)val.y * val.y;
    } else if constexpr (MODE == C1_ITER) {
      val = make_float2(0.f, 0.f);   // the update runs below, all loads first
    } else {  // C1_APPLY
      val = cscale(SRC[i], ok ? a.scale : 0.f);
    }
    pv[m] = val;
  }
  if constexpr (MODE == C1_ITER) {
    // finish iteration i-1 and start i: x += alpha p, r -= alpha q, p = r + beta p.
    // In chunks of H elements, every load of a chunk is issued before its first store.
    constexpr int H = VAH > 8 ? 8 : VAH;
    const bool xz = a.x_zero != 0;
#pragma unroll
    for (int m0 = 0; m0 < VAH; m0 += H) {
      float2 po[H], qo[H], ro[H], xo[H];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if (m0 + h >= VAH) break;
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
        if (m >= VAH) break;
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
  // Stockham rows of 512 and 768 points: the map row of coil c + 1 is loaded
  // into registers while coil c is transformed (measured: 512-point spiral
  // rows 6.63 -> 5.53 ms per application).  The two-step rows get their map
  // rows straight into the transform tiles, coil c + 1's once coil c's
  // transform is done; the short Stockham plans keep direct loads (their
  // many groups per wavefront would need more address registers than they
  // have).
  MapElem<ST> svn[CF::VMAX];
  auto load_maps = [&](int c) {
    const size_t moff = ((size_t)c * a.ny + y) * a.nx;
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      if (HALF && m >= VAH) continue;   // past the image row (zero)
      const int xx = CF::posA(lane, m);
      svn[m] = map_raw<ST>(a, moff + ((inA && xx < a.nx) ? xx : 0));
    }
  };
  if constexpr (PF) load_maps(0);
  for (int c = 0; c < a.nc; ++c) {
    float2 v[CF::VMAX];
    if constexpr (PF) {
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (HALF && m >= VAH) {   // past the image row
          v[m] = make_float2(0.f, 0.f);
          continue;
        }
        v[m] = cmul(widen(svn[m]), pv[m]);   // pv is 0 outside the row
      }
      if (c + 1 < a.nc) load_maps(c + 1);
    } else if constexpr (DMA) {
      wait_lds_loads();
      const ME* mrow = reinterpret_cast<const ME*>(lds);
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (HALF && m >= VAH) {   // past the image row
          v[m] = make_float2(0.f, 0.f);
          continue;
        }
        const int xx = CF::posA(lane, m);
        const bool ok = inA && xx < a.nx;
        v[m] = cmul(widen(mrow[ok ? xx : 0]), pv[m]);   // pv is 0 outside the row
      }
    } else {
      const size_t moff = ((size_t)c * a.ny + y) * a.nx;
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (HALF && m >= VAH) {   // past the image row
          v[m] = make_float2(0.f, 0.f);
          continue;
        }
        const int xx = CF::posA(lane, m);
        const bool ok = inA && xx < a.nx;
        v[m] = cmul(map_at<ST>(a, moff + (ok ? xx : 0)), pv[m]);   // pv is 0 outside the row
      }
    }
    CF::template forward<false>(v, lds, lane, tw);
    if constexpr (DMA) {
      if (c + 1 < a.nc) map_rows(c + 1);
    }
    if (active && inB) {
      const size_t off = (((size_t)k * a.nc + c) * a.ny + y) * a.Gx;
      if constexpr (ST == 2) {
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
// each, adjacent columns of one (k, c) plane.  HALF (the Toeplitz grids,
// ny = Gy / 2): the input column is zero past its first half and only the
// first half of the output is kept; both layouts place values m < VA / 2 and
// r < VB / 2 in the first half, so the zeros and the unused outputs are
// compile-time facts the compiler folds out of the first and last passes.
template <class CF, bool TB, bool HALF>
__global__ __launch_bounds__(256) void k_cols(Grid2dArgs a) {
  constexpr int L = CF::L, NGRP = 256 / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  constexpr int TS = NGRP + 1;  // padded tile row
  extern __shared__ float2 dyn[];
  // [ny][TS] tile; once every group holds its column in registers, the same
  // LDS serves as the NG exchange regions of the transforms
  float2* tile = dyn;
  float2* xch = dyn;
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  // Workgroups go to the eight XCDs in turn; workgroup b takes the strip at
  // v = (b mod 8) * ceil(W / 8) + b / 8 of the order (plane, strip), so each
  // XCD runs a contiguous run of strips and the cache lines that adjacent
  // strips share stay in one L2
  const long S = (a.Gx + NGRP - 1) / NGRP, W = S * (long)a.K * a.nc, per = (W + 7) / 8;
  const long vb = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (vb >= W) return;
  const int x0 = (int)(vb % S) * NGRP;
  const size_t plane = (size_t)(vb / S) * a.ny * a.Gx;
  const int ncol = min(NGRP, a.Gx - x0);
  if constexpr (TB) strip_load(tile, a.Tb + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
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
    if (HALF && m >= VA / 2) v[m] = make_float2(0.f, 0.f);
    else v[m] = (grp && inA && (HALF || yy < a.ny)) ? tile[yy * TS + g] : make_float2(0.f, 0.f);
  }
  __syncthreads();
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
    for (int m = 0; m < (HALF ? VA / 2 : VA); ++m) {
      const int yy = CF::posA(lane, m);
      if (HALF || yy < a.ny) tile[yy * TS + g] = v[m];
    }
  }
  __syncthreads();
  if constexpr (TB) strip_store(tile, a.Tb + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
  else strip_store(tile, a.T + plane + x0, a.ny, NGRP, TS, ncol, a.Gx);
}

// ---------------------------------------------------------------- row pass 2
template <class CF, int MODE, int ST, bool HALF>
__global__ __launch_bounds__(64) void k_rows_inv(Grid2dArgs a) {
  constexpr int L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  // HALF (the Toeplitz grids, nx = Gx / 2): only values m < VA / 2 of the
  // inverse transform lie in the image row
  constexpr int VAH = HALF ? VA / 2 : VA;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ double red[64 + L];   // lane 0 of a partial last group reads L entries
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
  constexpr bool DMA = CF::kRowsDma, PF = !DMA && CF::N >= 384;
  using TE = std::conditional_t<ST == 2, uint32_t, float2>;
  // two-step rows: coil c + 1's transformed rows go straight into the
  // transform tiles once coil c's inverse transform is done
  auto t_rows = [&](int c) {
    dma_rows<CF, TE, CF::SPAN * (int)(sizeof(float2) / sizeof(TE))>(reinterpret_cast<TE*>(lds_all), a.Gx, [&](int gi) {
      const long gq = (long)blockIdx.x * G + gi;
      const long gr = gq < (long)a.K * a.ny ? gq : 0;
      const size_t off = (((size_t)(gr / a.ny) * a.nc + c) * a.ny + (int)(gr % a.ny)) * a.Gx;
      if constexpr (ST == 2) return (const TE*)(a.Tb + off);
      else return (const TE*)(T + off);
    });
  };
  if constexpr (DMA) t_rows(0);
  // Stockham rows of 512 and 768 points: each coil's map rows come through LDS (a
  // buffer of their own, fetched when the coil starts and read after its
  // inverse transform); with the transformed row of the next coil already in
  // registers, the combine's own loads would be serialised for want of them
  using ME = MapElem<ST>;
  __shared__ ME mapbuf[PF ? G * CF::N : 1];
  auto map_rows = [&](int c) {
    dma_rows<CF, ME, CF::N>(mapbuf, a.nx, [&](int gi) {
      const long gq = (long)blockIdx.x * G + gi;
      const long gr = gq < (long)a.K * a.ny ? gq : 0;
      const size_t moff = ((size_t)c * a.ny + (int)(gr % a.ny)) * a.nx;
      if constexpr (ST >= 1) return (const ME*)(a.maps_bf + moff);
      else return (const ME*)(a.maps + moff);
    });
  };
  // p (or scale * src) of this row: lam p enters q first (when lam != 0); the
  // dots at the end load it again
  auto load_p = [&](float2* pa) {
#pragma unroll
    for (int m = 0; m < VA; ++m) {
      if (HALF && m >= VAH) continue;   // past the image row (zero)
      const int xx = CF::posA(lane, m);
      const bool ok = inA && xx < a.nx;
      const size_t i = rowoff + (ok ? xx : 0);
      const float2 raw = MODE == C1_APPLY ? SRC[i] : P[i];
      pa[m] = cscale(raw, ok ? (MODE == C1_APPLY ? a.scale : 1.f) : 0.f);
    }
  };
  float2 qa[CF::VMAX];
  if (a.lam != 0.f) {
    load_p(qa);
#pragma unroll
    for (int m = 0; m < VAH; ++m) qa[m] = cscale(qa[m], a.lam);
  } else {
#pragma unroll
    for (int m = 0; m < VAH; ++m) qa[m] = make_float2(0.f, 0.f);
  }
  // Stockham rows of 512 and 768 points: the transformed row of coil c + 1 is loaded
  // while coil c is inverted (raw storage form, unconditional loads from
  // in-row addresses; lanes outside layout B get zeros at use)
  TE tn[CF::VMAX];
  auto load_row = [&](int c) {
    const size_t off = (((size_t)k * a.nc + c) * a.ny + y) * a.Gx;
#pragma unroll
    for (int r = 0; r < VB; ++r) {
      const size_t j = off + (inB ? CF::posB(lane, r) : 0);
      if constexpr (ST == 2) tn[r] = a.Tb[j];
      else tn[r] = T[j];
    }
  };
  if constexpr (PF) load_row(0);
  for (int c = 0; c < a.nc; ++c) {
    float2 v[CF::VMAX];
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < VB; ++r) v[r] = widen(tn[r]);   // unused outside layout B
      map_rows(c);
      if (c + 1 < a.nc) load_row(c + 1);
    } else if constexpr (DMA) {
      wait_lds_loads();
      const TE* trow = reinterpret_cast<const TE*>(lds);
#pragma unroll   // lanes outside layout B read tile padding, unused by the transform
      for (int r = 0; r < VB; ++r) v[r] = widen(trow[CF::posB(lane, r)]);
    } else {
      const size_t off = (((size_t)k * a.nc + c) * a.ny + y) * a.Gx;
      if constexpr (ST == 2) {
#pragma unroll
        for (int r = 0; r < VB; ++r) v[r] = unpack_bf16x2(a.Tb[off + (inB ? CF::posB(lane, r) : 0)]);
      } else {
#pragma unroll
        for (int r = 0; r < VB; ++r) v[r] = T[off + (inB ? CF::posB(lane, r) : 0)];   // unused outside layout B
      }
    }
    CF::template inverse<true>(v, lds, lane, tw);
    if constexpr (DMA) {
      if (c + 1 < a.nc) t_rows(c + 1);
    }
    // the combine is unconditional (lanes outside the row are never stored
    // or summed)
    if constexpr (PF) {
      wait_lds_loads();
      const ME* mrow = mapbuf + (g < G ? g : 0) * CF::N;
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (HALF && m >= VAH) continue;   // past the image row (zero)
        const int xx = CF::posA(lane, m);
        const bool ok = inA && xx < a.nx;
        qa[m] = cadd(qa[m], cmulc(widen(mrow[ok ? xx : 0]), v[m]));
      }
    } else {
      const size_t moff = ((size_t)c * a.ny + y) * a.nx;
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (HALF && m >= VAH) continue;   // past the image row (zero)
        const int xx = CF::posA(lane, m);
        const bool ok = inA && xx < a.nx;
        qa[m] = cadd(qa[m], cmulc(map_at<ST>(a, moff + (ok ? xx : 0)), v[m]));
      }
    }
  }
  float2 pa[CF::VMAX], ra[CF::VMAX];
  load_p(pa);
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    if (HALF && m >= VAH) continue;   // past the image row (zero)
    const int xx = CF::posA(lane, m);
    const size_t i = rowoff + ((inA && xx < a.nx) ? xx : 0);
    ra[m] = MODE == C1_ITER ? R[i] : pa[m];
  }
  double d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
  for (int m = 0; m < VA; ++m) {
    if (HALF && m >= VAH) continue;   // past the image row (zero)
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
// Every row and column kernel holds at most two waves per SIMD here, so the
// plan per length is the one whose kernels fit 256 VGPRs without spilling:
// two-step plans (one LDS transpose per transform) where LA + VA values per
// lane fit, 32-lane groups for 576 and 640 points, and a 64-lane Stockham
// plan for 768 points (12 values per lane; the 32-lane plans of 768 points
// spill).  Measured per normal-operator application against the 16- and
// 32-lane Stockham plans they replace: 288-point grid 6.87 -> 2.55 ms (30
// coils, K = 128), 576 x 576 6.23 -> 3.54 ms and 640 x 640 4.82 -> 3.26 ms
// (spiral, K = 64), 768 x 768 13.4 -> 6.6 ms (32 coils, K = 32); 160- and
// 192-point grids (16 coils, K = 256) 1.03 -> 0.86 and 1.44 -> 1.15 ms.  The
// 64-lane plan of 512 points (8 x 8 x 8) measured 2 % slower than the 32-lane
// one, and the two-step plans of 96 and 128 points 5-15 % slower than the
// Stockham ones kept there.
using L64 = TwoStep<8, 8>;
using L96 = StockhamCol<FFTPlan<96, 8, 12, 4, 2>>;
using L128 = StockhamCol<FFTPlan<128, 16, 8, 4, 4>>;
using L160 = TwoStep<16, 10>;
using L192 = TwoStep<16, 12>;
using L256 = TwoStep<16, 16>;
using L288 = TwoStep<18, 16>;
using L320 = TwoStep<20, 16>;
using L384 = TwoStep<24, 16>;
using L512 = StockhamCol<FFTPlan<512, 32, 16, 16, 2>>;
using L576 = TwoStep<32, 18>;
using L640 = TwoStep<32, 20>;
using L768 = StockhamCol<FFTPlan<768, 64, 12, 4, 4, 4>>;

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

template <class CF, int ST, bool HALF>
static hipError_t rows_fwd_h(int mode, const Grid2dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  const long rows = (long)a.K * a.ny;
  dim3 grid((unsigned)((rows + G - 1) / G)), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL((k_rows_fwd<CF, C1_FIRST_PROBE, ST, HALF>), grid, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL((k_rows_fwd<CF, C1_FIRST_BUF, ST, HALF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_rows_fwd<CF, C1_ITER, ST, HALF>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_rows_fwd<CF, C1_APPLY, ST, HALF>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class CF, int ST, bool HALF>
static hipError_t rows_inv_h(int mode, const Grid2dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  const long rows = (long)a.K * a.ny;
  dim3 grid((unsigned)((rows + G - 1) / G)), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: case C1_FIRST_BUF:
      hipLaunchKernelGGL((k_rows_inv<CF, C1_FIRST_BUF, ST, HALF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_rows_inv<CF, C1_ITER, ST, HALF>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_rows_inv<CF, C1_APPLY, ST, HALF>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the half-row variants when the image row is the first half of the grid row
// (the Toeplitz grids, nx = Gx / 2)
template <class CF, int ST>
static hipError_t rows_fwd(int mode, const Grid2dArgs& a, hipStream_t s) {
  if constexpr (CF::VA % 2 == 0) {
    if (2 * a.nx == a.Gx) return rows_fwd_h<CF, ST, true>(mode, a, s);
  }
  return rows_fwd_h<CF, ST, false>(mode, a, s);
}

template <class CF, int ST>
static hipError_t rows_inv(int mode, const Grid2dArgs& a, hipStream_t s) {
  if constexpr (CF::VA % 2 == 0) {
    if (2 * a.nx == a.Gx) return rows_inv_h<CF, ST, true>(mode, a, s);
  }
  return rows_inv_h<CF, ST, false>(mode, a, s);
}

template <class CF, bool TB, bool HALF>
static hipError_t cols_launch(const Grid2dArgs& a, size_t lds, hipStream_t s) {
  constexpr int NGRP = 256 / CF::L;
  // allow more than the default 64 KiB of dynamic LDS (once per process,
  // thread-safe initialisation)
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_cols<CF, TB, HALF>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  const long W = (long)((a.Gx + NGRP - 1) / NGRP) * a.K * a.nc;
  dim3 grid((unsigned)(8 * ((W + 7) / 8))), block(256);
  hipLaunchKernelGGL((k_cols<CF, TB, HALF>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <class CF, bool TB>
static hipError_t cols(const Grid2dArgs& a, hipStream_t s) {
  constexpr int L = CF::L, NGRP = 256 / L, NG = (256 + L - 1) / L;
  const size_t lds = std::max((size_t)a.ny * (NGRP + 1), (size_t)NG * CF::SPAN) * sizeof(float2);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if constexpr (CF::VA % 2 == 0 && CF::VB % 2 == 0) {
    if (2 * a.ny == a.Gy) return cols_launch<CF, TB, true>(a, lds, s);
  }
  return cols_launch<CF, TB, false>(a, lds, s);
}


// One application of the normal operator (three passes) with storage ST:
// 0 complex64, 1 bfloat16 maps, 2 bfloat16 maps and planes
template <int ST>
static hipError_t grid_normal(int mode, const Grid2dArgs& a, hipStream_t s) {
  hipError_t e = with_line(a.Gx, [&](auto cf) { return rows_fwd<decltype(cf), ST>(mode, a, s); });
  if (e != hipSuccess) return e;
  e = with_line(a.Gy, [&](auto cf) { return cols<decltype(cf), ST == 2>(a, s); });
  if (e != hipSuccess) return e;
  return with_line(a.Gx, [&](auto cf) { return rows_inv<decltype(cf), ST>(mode, a, s); });
}

}  // namespace pico
