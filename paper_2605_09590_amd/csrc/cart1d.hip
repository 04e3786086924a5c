// Separable Cartesian SENSE normal operator and the CG building blocks.
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
#include "fft.h"
#include "runtime.h"

namespace pico {

// q = (M + lam) p for one probe column held in layout A by the lanes of one
// group: per coil, S' p -> FFT (layout A -> B) -> weight mask[k]/ny -> inverse
// FFT (B -> A) -> accumulate conj(S') times the result.
template <class CF>
__device__ __forceinline__ void normal_col(const float2 (&pv)[CF::VMAX], float2 (&qa)[CF::VMAX],
                                           float lam, MapRef mcol, int nc,
                                           uint32_t mbits, float2* lds, int lane,
                                           const typename CF::Tw& tw) {
  constexpr int N = CF::N;
  constexpr float minv = 1.0f / N;
  const bool inA = CF::inA(lane);
#pragma unroll
  for (int m = 0; m < CF::VA; ++m) qa[m] = cscale(pv[m], lam);
  for (int c = 0; c < nc; ++c) {
    const MapRef s = mcol + (size_t)c * N;
    float2 v[CF::VMAX];
#pragma unroll
    for (int m = 0; m < CF::VA; ++m) v[m] = inA ? cmul(s[CF::posA(lane, m)], pv[m]) : make_float2(0.f, 0.f);
    CF::template forward<false>(v, lds, lane, tw);
#pragma unroll
    for (int r = 0; r < CF::VB; ++r)
      v[r] = ((mbits >> r) & 1u) ? cscale(v[r], minv) : make_float2(0.f, 0.f);
    CF::template inverse<true>(v, lds, lane, tw);
    if (inA) {
#pragma unroll
      for (int m = 0; m < CF::VA; ++m) qa[m] = cadd(qa[m], cmulc(s[CF::posA(lane, m)], v[m]));
    }
  }
}

// Sum of one double per lane over each lane group of L lanes, in lane order
// (bitwise reproducible); the result is valid in the group's first lane.
template <int L>
__device__ __forceinline__ double group_reduce(double v, double* red, int lane) {
  red[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (lane == 0) {
    const int base = threadIdx.x;
    for (int i = 0; i < L; ++i) s += red[base + i];
  }
  __syncthreads();
  return s;
}

template <class CF, int MODE>
__global__ __launch_bounds__(64) void k_cart1d(Cart1dArgs a) {
  constexpr int N = CF::N, L = CF::L, G = 64 / L, NG = (64 + L - 1) / L;
  constexpr int VA = CF::VA, VB = CF::VB;
  __shared__ float2 lds_all[NG * CF::SPAN];
  __shared__ double red[64];
  const int g = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  const int col = blockIdx.y;
  const int k = blockIdx.x * G + g;
  const bool active = g < G && k < a.K;
  const int kk = active ? k : 0;  // idle lanes work on probe 0 but never store
  const bool inA = CF::inA(lane), inB = CF::inB(lane);
  float2* lds = lds_all + g * CF::SPAN;

  typename CF::Tw tw;
  CF::load_tw(tw, a.twt, lane);
  uint32_t mbits = 0;
  if (inB) {
#pragma unroll
    for (int r = 0; r < VB; ++r) mbits |= (a.maskw[CF::posB(lane, r)] != 0.f ? 1u : 0u) << r;
  }

  const size_t base = ((size_t)kk * a.nx + col) * N;
  const MapRef mcol = MapRef{a.maps, a.maps_bf} + (size_t)col * a.nc * N;
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
        if ((mbits >> r) & 1u) {
          const uint32_t elem = (uint32_t)(((size_t)c * N + kc) * a.nx + col);
          const float2 n = draw_probe(a.seed, a.first + kk, elem, 1u, 3);
          v[r] = cscale(n, ((kc + N / 2) & 1) ? -rs : rs);
        } else {
          v[r] = make_float2(0.f, 0.f);
        }
      }
      CF::template inverse<true>(v, lds, lane, tw);
      const MapRef s = mcol + (size_t)c * N;
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
    d0 = group_reduce<L>(d0, red, lane);
    if (active && lane == 0) a.part[((size_t)k * a.nx + col) * 4] = d0;
    return;
  } else {
    // rv keeps r_i for the d3 = Re(r^H q) partial; pv = p_i enters the normal operator
    float2 rv[CF::VMAX];
    if (inA) {
      if constexpr (MODE == C1_FIRST_PROBE) {
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          const int y = CF::posA(lane, m);
          pv[m] = draw_probe(a.seed, a.first + kk, (uint32_t)(y * a.nx + col), 0u, a.dist);
          rv[m] = pv[m];
          if (active) { a.r[base + y] = pv[m]; a.p[base + y] = pv[m]; }
        }
      } else if constexpr (MODE == C1_FIRST_BUF) {
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          const int y = CF::posA(lane, m);
          pv[m] = a.r[base + y];
          rv[m] = pv[m];
          if (active) a.p[base + y] = pv[m];
        }
      } else if constexpr (MODE == C1_ITER) {
        // finish iteration i-1 and start iteration i:
        //   x += alpha p, r -= alpha q, p = r + beta p
        const float alpha = (float)a.alpha[kk];
        const float beta = (float)a.beta[kk];
#pragma unroll
        for (int m = 0; m < VA; ++m) {
          const int y = CF::posA(lane, m);
          const float2 po = a.p[base + y];
          const float2 qo = a.q[base + y];
          const float2 xo = a.x_zero ? make_float2(0.f, 0.f) : a.x[base + y];
          rv[m] = cfma(a.r[base + y], -alpha, qo);
          pv[m] = cfma(rv[m], beta, po);
          if (active) {
            a.x[base + y] = cfma(xo, alpha, po);
            a.r[base + y] = rv[m];
            a.p[base + y] = pv[m];
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
    normal_col<CF>(pv, qa, a.lam, mcol, a.nc, mbits, lds, lane, tw);

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
    d0 = group_reduce<L>(d0, red, lane);
    d1 = group_reduce<L>(d1, red, lane);
    d2 = group_reduce<L>(d2, red, lane);
    d3 = group_reduce<L>(d3, red, lane);
    if (active && lane == 0) {
      double* pp = a.part + ((size_t)k * a.nx + col) * 4;
      pp[0] = d0;
      pp[1] = d1;
      pp[2] = d2;
      pp[3] = d3;
    }
  }
}

// ------------------------------------------------------------ dispatch
template <class CF>
static hipError_t launch_plan(int mode, const Cart1dArgs& a, hipStream_t s) {
  constexpr int G = 64 / CF::L;
  dim3 grid((a.K + G - 1) / G, a.nx), block(64);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL((k_cart1d<CF, C1_FIRST_PROBE>), grid, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL((k_cart1d<CF, C1_FIRST_BUF>), grid, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL((k_cart1d<CF, C1_ITER>), grid, block, 0, s, a); break;
    case C1_APPLY: hipLaunchKernelGGL((k_cart1d<CF, C1_APPLY>), grid, block, 0, s, a); break;
    case C1_PMR_RHS: hipLaunchKernelGGL((k_cart1d<CF, C1_PMR_RHS>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Column-FFT layouts per line length.  Stockham plans keep N/T values on T
// lanes through every pass; two-step plans split N = LA * VA over LA lanes
// with a single LDS transpose per transform.
using Col64 = TwoStep<8, 8>;
using Col96 = StockhamCol<FFTPlan<96, 8, 12, 4, 2>>;
using Col128 = StockhamCol<FFTPlan<128, 16, 8, 4, 4>>;
using Col160 = StockhamCol<FFTPlan<160, 8, 20, 4, 2>>;
using Col192 = StockhamCol<FFTPlan<192, 16, 12, 4, 4>>;
using Col256 = TwoStep<16, 16>;
using Col288 = StockhamCol<FFTPlan<288, 16, 18, 2, 2, 2, 2>>;
using Col320 = TwoStep<20, 16>;
using Col384 = StockhamCol<FFTPlan<384, 16, 24, 4, 4>>;
using Col512 = StockhamCol<FFTPlan<512, 32, 16, 16, 2>>;

bool cart1d_supported(int ny) {
  switch (ny) {
    case 64: case 96: case 128: case 160: case 192: case 256: case 288: case 320: case 384: case 512:
      return true;
    default:
      return false;
  }
}

hipError_t launch_cart1d(int mode, const Cart1dArgs& a, hipStream_t s) {
  switch (a.ny) {
    case 64: return launch_plan<Col64>(mode, a, s);
    case 96: return launch_plan<Col96>(mode, a, s);
    case 128: return launch_plan<Col128>(mode, a, s);
    case 160: return launch_plan<Col160>(mode, a, s);
    case 192: return launch_plan<Col192>(mode, a, s);
    case 256: return launch_plan<Col256>(mode, a, s);
    case 288: return launch_plan<Col288>(mode, a, s);
    case 320: return launch_plan<Col320>(mode, a, s);
    case 384: return launch_plan<Col384>(mode, a, s);
    case 512: return launch_plan<Col512>(mode, a, s);
    default: return hipErrorInvalidValue;
  }
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
      const float2 v = draw_probe(a.seed, a.first + k, vox, 0u, a.dist);
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
