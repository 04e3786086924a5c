// Separable Cartesian SENSE normal operator (kernel templates; complex64 and
// bfloat16 map storage are instantiated in translation units of their own).
//
// With a phase-encode mask that is constant along kx, the whitened normal
// operator M = sum_c S_c^H F^H P F S_c (Sec. 2.1, Eqs. (3), (6)) is block
// diagonal over image columns: F_x^H F_x = I cancels, leaving one 1-D
// transform along y per column and coil.  For even ny the centred
// orthonormal DFT (fftshift o fft o ifftshift) equals (-1)^(ny/2) D F D / sqrt(ny)
// with D = diag((-1)^y) and F the plain DFT, so F_c^H P F_c = D F^H P F D / ny:
// D is folded into the whitened maps once, the centred-order mask applies
// unchanged, and each coil costs one forward and one inverse unnormalised
// FFT with the weight mask[k] / ny in between.
//
// Layout: every per-probe field is stored column-major, [K][nx][ny], so a
// column is one contiguous line; maps are [nx][nc][ny].  One workgroup is one
// wavefront holding G = 64/L probe columns of the same image column; each
// column FFT lives in the registers of a group of L lanes and exchanges
// through LDS.
#pragma once

#include <type_traits>

#include "fft.h"
#include "runtime.h"

namespace pico {
// Coil maps of one column: complex64, or packed bfloat16 pairs
struct MapsF32 {
  const float2* p;
  static __device__ __forceinline__ MapsF32 of(const Cart1dArgs& a) { return MapsF32{a.maps}; }
  __device__ __forceinline__ float2 operator[](size_t i) const { return p[i]; }
  __device__ __forceinline__ MapsF32 operator+(size_t o) const { return MapsF32{p + o}; }
};
struct MapsBf16 {
  const uint32_t* p;
  static __device__ __forceinline__ MapsBf16 of(const Cart1dArgs& a) { return MapsBf16{a.maps_bf}; }
  __device__ __forceinline__ float2 operator[](size_t i) const { return unpack_bf16x2(p[i]); }
  __device__ __forceinline__ MapsBf16 operator+(size_t o) const { return MapsBf16{p + o}; }
};


// Mask weights mask[k] / ny of a lane's layout-B lines.  Two-step plans keep
// them in registers (one multiply per value); the Stockham plans, whose
// registers are full, keep one bit per line and select.
template <class CF>
struct MaskLines {
  static constexpr bool kRegs = CF::kMaskInRegs;
  float w[kRegs ? CF::VB : 1];
  uint32_t bits = 0;
  __device__ __forceinline__ void load(const float* __restrict__ maskw, int lane) {
    const bool inB = CF::inB(lane);
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) {
      // one batch of loads from in-bounds indices, zeroed by a factor (a
      // load under the lane condition gets a branch and a wait of its own)
      const float m = maskw[inB ? CF::posB(lane, r) : 0] * (inB ? 1.f : 0.f);
      if constexpr (kRegs) w[r] = m;
      bits |= (m != 0.f ? 1u : 0u) << r;
    }
  }
  __device__ __forceinline__ bool on(int r) const { return (bits >> r) & 1u; }
  __device__ __forceinline__ float2 apply(float2 v, int r) const {
    if constexpr (kRegs) return cscale(v, w[r]);
    else return on(r) ? cscale(v, 1.0f / CF::N) : make_float2(0.f, 0.f);
  }
};

// Coil map columns of one image column, staged through LDS: the wavefront's
// probe groups all work on the same image column, so its 64 lanes load each
// coil's column once (N / 64 values per lane) into one of two LDS buffers,
// the next coil's while the current one is transformed.  Plans whose
// registers are full read the maps from global memory directly.
template <class CF, class MS>
struct MapCols {
  static constexpr int N = CF::N;
  static constexpr bool kLds = CF::kMapsInLds;
  static constexpr int NPL = kLds ? (N + 63) / 64 : 1;   // values per wave lane
  static constexpr int LDS = kLds ? 2 * N : 1;           // float2, two buffers
  MS mcol;
  float2* buf;
  float2 pre[NPL];
  __device__ __forceinline__ void fetch(int c) {   // global loads of coil c (kept in flight)
    if constexpr (kLds) {
      const MS s = mcol + (size_t)c * N;
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int i = (int)threadIdx.x + 64 * j;
        if (N % 64 == 0 || i < N) pre[j] = s[i];
      }
    }
  }
  __device__ __forceinline__ void stash(int c) {   // coil c's values into its buffer
    if constexpr (kLds) {
      float2* b = buf + (c & 1) * N;
#pragma unroll
      for (int j = 0; j < NPL; ++j) {
        const int i = (int)threadIdx.x + 64 * j;
        if (N % 64 == 0 || i < N) b[i] = pre[j];
      }
    }
  }
  __device__ __forceinline__ float2 at(int c, int y) const {
    if constexpr (kLds) return buf[(c & 1) * N + y];
    else return (mcol + (size_t)c * N)[y];
  }
};

// q = (M + lam) p for one probe column held in layout A by the lanes of one
// group: per coil, S' p -> FFT (layout A -> B) -> weight mask[k]/ny -> inverse
// FFT (B -> A) -> accumulate conj(S') times the result.  With the maps in LDS,
// coil c + 1's column is loaded during coil c's forward transform and stored
// between the two transforms: its buffer was last read by coil c - 1 (before
// the forward transform's barriers), and the inverse transform's barriers
// publish it before coil c + 1 reads it.
template <class CF, class MS>
__device__ __forceinline__ void normal_col(const float2 (&pv)[CF::VMAX], float2 (&qa)[CF::VMAX],
                                           float lam, MapCols<CF, MS>& mc, int nc,
                                           const MaskLines<CF>& mk, float2* lds, int lane,
                                           const typename CF::Tw& tw) {
  const bool inA = CF::inA(lane);
#pragma unroll
  for (int m = 0; m < CF::VA; ++m) qa[m] = cscale(pv[m], lam);
  if constexpr (MapCols<CF, MS>::kLds) {   // coil 0's loads were issued by the caller
    mc.stash(0);
    __syncthreads();
  }
  for (int c = 0; c < nc; ++c) {
    if (c + 1 < nc) mc.fetch(c + 1);
    float2 v[CF::VMAX];
#pragma unroll
    for (int m = 0; m < CF::VA; ++m) v[m] = inA ? cmul(mc.at(c, CF::posA(lane, m)), pv[m]) : make_float2(0.f, 0.f);
    CF::template forward<false>(v, lds, lane, tw);
#pragma unroll
    for (int r = 0; r < CF::VB; ++r) v[r] = mk.apply(v[r], r);
    if (c + 1 < nc) mc.stash(c + 1);
    CF::template inverse<true>(v, lds, lane, tw);
    if (inA) {
#pragma unroll
      for (int m = 0; m < CF::VA; ++m) qa[m] = cadd(qa[m], cmulc(mc.at(c, CF::posA(lane, m)), v[m]));
    }
  }
}

// Sums of J doubles per lane over each lane group of L lanes, each in lane
// order (bitwise reproducible): lane j < J of the group returns sum j.  red
// holds (64 + L) J doubles (a partial last group reads past the wavefront).
template <int L, int J>
__device__ __forceinline__ double group_reduce(const double (&v)[J], double* red, int lane) {
#pragma unroll
  for (int j = 0; j < J; ++j) red[threadIdx.x * J + j] = v[j];
  __syncthreads();
  double s = 0.0;
  if (lane < J) {
    const int base = (threadIdx.x - lane) * J + lane;
    for (int i = 0; i < L; ++i) s += red[base + i * J];
  }
  __syncthreads();
  return s;
}

template <class CF, int MODE, bool BF>
__global__ __launch_bounds__(64) void k_cart1d(Cart1dArgs a) {
  constexpr int N = CF::N, L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  using MS = std::conditional_t<BF, MapsBf16, MapsF32>;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ float2 lds_maps[MapCols<CF, MS>::LDS];
  // the partial-dot reduction reuses the transform's LDS once it is done
  static_assert(NG * CF::SPAN * sizeof(float2) >= (64 + L) * 4 * sizeof(double), "reduction space");
  double* red = reinterpret_cast<double*>(lds_all);
  const int g = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  const int col = blockIdx.y;
  const int k = blockIdx.x * G + g;
  const bool active = g < G && k < a.K;
  const int kk = active ? k : 0;  // idle lanes work on probe 0 but never store
  const bool inA = CF::inA(lane);
  float2* lds = lds_all + g * CF::SPAN;

  typename CF::Tw tw;
  CF::load_tw(tw, a.twt, lane);
  MaskLines<CF> mk;
  mk.load(a.maskw, lane);

  const size_t base = ((size_t)kk * a.nx + col) * N;
  const MS mcol = MS::of(a) + (size_t)col * a.nc * N;
  float2 pv[CF::VMAX];
  double d0 = 0.0;

  if constexpr (MODE == C1_PMR_RHS) {
    // r = A^H n = sum_c conj(S_w,c) F_c^H P n_c with F_c^H = (-1)^(ny/2) D F^H D / sqrt(ny):
    // per coil, w[k] = (-1)^(ny/2 + k) n[k] / sqrt(ny) on the sampled lines,
    // unnormalised inverse FFT, times conj(S') (D already folded into S').
    const float rs = rsqrtf((float)N);
#pragma unroll
    for (int m = 0; m < VA; ++m) pv[m] = make_float2(0.f, 0.f);
    for (int c = 0; c < a.nc; ++c) {
      float2 v[CF::VMAX];
#pragma unroll
      for (int r = 0; r < VB; ++r) {
        const int kc = CF::posB(lane, r);
        if (mk.on(r)) {
          const uint32_t elem = (uint32_t)(((size_t)c * N + kc) * a.nx + col);
          const float2 n = draw_probe(arg_seed(a), arg_first(a) + kk, elem, 1u, 3);
          v[r] = cscale(n, ((kc + N / 2) & 1) ? -rs : rs);
        } else {
          v[r] = make_float2(0.f, 0.f);
        }
      }
      CF::template inverse<true>(v, lds, lane, tw);
      const MS s = mcol + (size_t)c * N;
      if (inA) {
#pragma unroll
        for (int m = 0; m < VA; ++m) pv[m] = cadd(pv[m], cmulc(s[CF::posA(lane, m)], v[m]));
      }
    }
    if (inA) {
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (active) a.r[base + CF::posA(lane, m)] = pv[m];
        d0 += (double)pv[m].x * pv[m].x + (double)pv[m].y * pv[m].y;
      }
    }
    const double dd[1] = {d0};
    d0 = group_reduce<L, 1>(dd, red, lane);
    if (active && lane == 0) a.part[((size_t)k * a.nx + col) * 4] = d0;
    return;
  } else {
    // coil 0's map column is loaded while the CG vectors are
    MapCols<CF, MS> mc;
    mc.mcol = mcol;
    mc.buf = lds_maps;
    mc.fetch(0);
    // rv keeps r_i for the d3 = Re(r^H q) partial; pv = p_i enters the normal operator
    float2 rv[CF::VMAX];
    if (inA) {
      if constexpr (MODE == C1_FIRST_PROBE) {
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          const int y = CF::posA(lane, m);
          pv[m] = draw_probe(arg_seed(a), arg_first(a) + kk, (uint32_t)(y * a.nx + col), 0u, a.dist);
          rv[m] = pv[m];
          if (active) { a.r[base + y] = pv[m]; a.p[base + y] = pv[m]; }
        }
      } else if constexpr (MODE == C1_FIRST_BUF) {
        const float2* __restrict__ R = a.r;   // all loads before the first store
        float2* __restrict__ P = a.p;
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          pv[m] = R[base + CF::posA(lane, m)];
          rv[m] = pv[m];
        }
        if (active) {
#pragma unroll
          for (int m = 0; m < VA; ++m) P[base + CF::posA(lane, m)] = pv[m];
        }
      } else if constexpr (MODE == C1_ITER) {
        // finish iteration i-1 and start iteration i:
        //   x += alpha p, r -= alpha q, p = r + beta p
        // The fields never alias one another: restrict lets every load of a
        // chunk of H elements go out before the chunk's first store (else
        // each element's loads wait behind the previous element's stores).
        float2* __restrict__ X = a.x;
        float2* __restrict__ R = a.r;
        float2* __restrict__ P = a.p;
        const float2* __restrict__ Q = a.q;
        const float alpha = (float)a.alpha[kk];
        const float beta = (float)a.beta[kk];
        const bool xz = a.x_zero != 0;
        constexpr int H = VA > 8 ? 8 : VA;
#pragma unroll
        for (int m0 = 0; m0 < VA; m0 += H) {
          float2 po[H], qo[H], ro[H], xo[H];
#pragma unroll
          for (int h = 0; h < H; ++h) {
            if (m0 + h >= VA) break;
            const size_t i = base + CF::posA(lane, m0 + h);
            po[h] = P[i];
            qo[h] = Q[i];
            ro[h] = R[i];
            xo[h] = X[i];
          }
#pragma unroll
          for (int h = 0; h < H; ++h) {
            const int m = m0 + h;
            if (m >= VA) break;
            const size_t i = base + CF::posA(lane, m);
            rv[m] = cfma(ro[h], -alpha, qo[h]);
            pv[m] = cfma(rv[m], beta, po[h]);
            if (active) {
              X[i] = cfma(xz ? make_float2(0.f, 0.f) : xo[h], alpha, po[h]);
              R[i] = rv[m];
              P[i] = pv[m];
            }
          }
        }
      } else {  // C1_APPLY
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          pv[m] = cscale(a.src[base + CF::posA(lane, m)], a.scale);
          rv[m] = make_float2(0.f, 0.f);
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        pv[m] = make_float2(0.f, 0.f);
        rv[m] = make_float2(0.f, 0.f);
      }
    }

    float2 qa[CF::VMAX];
    normal_col<CF, MS>(pv, qa, a.lam, mc, a.nc, mk, lds, lane, tw);

    double d1 = 0.0, d2 = 0.0, d3 = 0.0;
    if (inA) {
#pragma unroll
      for (int m = 0; m < VA; ++m) {
        if (active) a.q[base + CF::posA(lane, m)] = qa[m];
        d0 += (double)rv[m].x * rv[m].x + (double)rv[m].y * rv[m].y;
        d1 += (double)pv[m].x * qa[m].x + (double)pv[m].y * qa[m].y;
        d2 += (double)qa[m].x * qa[m].x + (double)qa[m].y * qa[m].y;
        d3 += (double)rv[m].x * qa[m].x + (double)rv[m].y * qa[m].y;
      }
    }
    const double dd[4] = {d0, d1, d2, d3};
    const double sj = group_reduce<L, 4>(dd, red, lane);
    if (active && lane < 4) a.part[((size_t)k * a.nx + col) * 4 + lane] = sj;
  }
}

// ------------------------------------------------------------ dispatch
template <class CF, bool BF>
static hipError_t launch_plan(int mode, const Cart1dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  dim3 grid((a.K + G - 1) / G, a.nx), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL((k_cart1d<CF, C1_FIRST_PROBE, BF>), grid, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL((k_cart1d<CF, C1_FIRST_BUF, BF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_cart1d<CF, C1_ITER, BF>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_cart1d<CF, C1_APPLY, BF>), grid, block, 0, s, a); break;
    case C1_PMR_RHS: hipLaunchKernelGGL((k_cart1d<CF, C1_PMR_RHS, BF>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Column-FFT layouts per line length.  Stockham plans keep N/T values on T
// lanes through every pass; two-step plans split N = LA * VA over LA lanes
// with a single LDS transpose per transform.  Each length takes the faster
// plan measured (K = 256, 16 coils, ms per application, replaced Stockham
// plan first): 128 points 0.192 -> 0.152, 160 0.560 -> 0.225 (that plan
// spilled), 192 0.398 -> 0.312, 288 2.93 -> 0.77 and 384 5.22 -> 1.42 (16
// lanes with 18 and 24 values each: one wave per SIMD, spilled), 512 4.87 ->
// 2.08 (32 lanes with 16 values -> 64 lanes with 8); at 96 points the
// Stockham plan stays (0.132 against 0.201 for two-step 8 x 12).
using Col64 = TwoStep<8, 8>;
using Col96 = StockhamCol<FFTPlan<96, 8, 12, 4, 2>>;
using Col128 = TwoStep<16, 8>;
using Col160 = TwoStep<16, 10>;
using Col192 = TwoStep<16, 12>;
using Col256 = TwoStep<16, 16>;
using Col288 = TwoStep<18, 16>;
using Col320 = TwoStep<20, 16>;
using Col384 = TwoStep<24, 16>;
using Col512 = StockhamCol<FFTPlan<512, 64, 8, 8, 8>>;


template <bool BF>
static hipError_t cart1d_dispatch(int mode, const Cart1dArgs& a, hipStream_t s) {
  switch (a.ny) {
    case 64: return launch_plan<Col64, BF>(mode, a, s);
    case 96: return launch_plan<Col96, BF>(mode, a, s);
    case 128: return launch_plan<Col128, BF>(mode, a, s);
    case 160: return launch_plan<Col160, BF>(mode, a, s);
    case 192: return launch_plan<Col192, BF>(mode, a, s);
    case 256: return launch_plan<Col256, BF>(mode, a, s);
    case 288: return launch_plan<Col288, BF>(mode, a, s);
    case 320: return launch_plan<Col320, BF>(mode, a, s);
    case 384: return launch_plan<Col384, BF>(mode, a, s);
    case 512: return launch_plan<Col512, BF>(mode, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pico
