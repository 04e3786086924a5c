// Compressed-sensing reconstruction (FISTA with an L1 penalty on a 4-level
// periodised db4 wavelet transform) and its forward-mode Jacobian probes.
//
// Primal, once per operator (step 1 of the normalised problem, Sec. 3.3):
//   z_k = y_k - (M y_k - A^H b) / s^2,  c_k = Psi z_k (stored),
//   x_k = Psi^H soft_lam(c_k),  y_{k+1} = x_k + theta_k (x_k - x_{k-1}).
// Tangent for K probes w at once (Sec. 2.2, CS extension: u = J w):
//   zd = yd - (M yd - A^H w) / s^2,  xd = Psi^H D_k(Psi zd),
//   yd' = xd + theta_k (xd - xd_prev),  accumulate |xd_T|^2.
// D_k is the derivative of complex soft-thresholding at the stored c_k:
//   |c| > lam: d = dc - (lam/|c|) c^ j Im(conj(c^) dc), c^ = c/|c|;  else 0;
//   lam = 0: identity.  Only detail coefficients are thresholded.
//
// Wavelet: orthonormal, periodised; analysis a[i] = sum_k h[k] x[(2i+k) mod n],
// d[i] = sum_k g[k] x[(2i+k) mod n], g[k] = (-1)^k h[7-k], stored [a | d];
// rows then columns of the current low-pass block per level.
#include "device_common.h"
#include "runtime.h"

#include <algorithm>
#include <vector>

namespace pico {

// Daubechies' extremal-phase scaling filter with 4 vanishing moments
// (8 taps; Daubechies, "Ten Lectures on Wavelets", Table 6.1, N = 4).
#define PICO_DB4_TAPS                                                                     \
  0.2303778133088964, 0.7148465705529154, 0.6308807679298587, -0.0279837694168599,      \
      -0.1870348117190931, 0.0308413818355607, 0.0328830116668852, -0.0105974017850690
__constant__ float c_h32[8] = {PICO_DB4_TAPS};
__constant__ double c_h64[8] = {PICO_DB4_TAPS};

template <class R> __device__ __forceinline__ R wav_h(int k);
template <> __device__ __forceinline__ float wav_h<float>(int k) { return c_h32[k]; }
template <> __device__ __forceinline__ double wav_h<double>(int k) { return c_h64[k]; }
template <class R> __device__ __forceinline__ R wav_g(int k) {
  return (k & 1) ? -wav_h<R>(7 - k) : wav_h<R>(7 - k);
}

// complex (float2 / double2) accumulate acc + s * v with a real tap s
__device__ __forceinline__ double2 cfma(double2 acc, double s, double2 a) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}
template <class C> struct Real;
template <> struct Real<float2> { using T = float; };
template <> struct Real<double2> { using T = double; };
template <class C> __device__ __forceinline__ C czero() { C z; z.x = 0; z.y = 0; return z; }

// Derivative of complex soft-thresholding at the stored coefficient c (FP64,
// the active-set decision in FP64) applied to the tangent d:
//   |c| > lam: d - (lam / |c|) c^ j Im(conj(c^) d), c^ = c / |c|;  else 0.
__device__ __forceinline__ float2 dsoft_one(float2 d, double2 c, double lam) {
  const double a = sqrt(c.x * c.x + c.y * c.y);
  if (!(a > lam)) return make_float2(0.f, 0.f);
  const float chx = (float)(c.x / a), chy = (float)(c.y / a);
  const float im = chx * d.y - chy * d.x;        // Im(conj(c^) d)
  const float f = (float)(lam / a) * im;         // d - f * j * c^
  return make_float2(d.x + f * chy, d.y - f * chx);
}

// analysis along x of the block [by][bx] of each image
template <class C>
__global__ void k_dwt_x(const C* __restrict__ in, C* __restrict__ out, int ny, int nx, int by, int bx) {
  using R = typename Real<C>::T;
  const int half = bx / 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)by * half) return;
  const int y = (int)(t / half), i = (int)(t % half);
  const size_t img = (size_t)blockIdx.y * ny * nx;
  const C* row = in + img + (size_t)y * nx;
  C a = czero<C>(), d = czero<C>();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const C v = row[(2 * i + k) % bx];
    a = cfma(a, wav_h<R>(k), v);
    d = cfma(d, wav_g<R>(k), v);
  }
  out[img + (size_t)y * nx + i] = a;
  out[img + (size_t)y * nx + half + i] = d;
}

// analysis along y
template <class C>
__global__ void k_dwt_y(const C* __restrict__ in, C* __restrict__ out, int ny, int nx, int by, int bx) {
  using R = typename Real<C>::T;
  const int half = by / 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)half * bx) return;
  const int j = (int)(t / bx), x = (int)(t % bx);
  const size_t img = (size_t)blockIdx.y * ny * nx;
  C a = czero<C>(), d = czero<C>();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const C v = in[img + (size_t)((2 * j + k) % by) * nx + x];
    a = cfma(a, wav_h<R>(k), v);
    d = cfma(d, wav_g<R>(k), v);
  }
  out[img + (size_t)j * nx + x] = a;
  out[img + (size_t)(half + j) * nx + x] = d;
}

// synthesis along y: x[m] = sum over taps k = m (mod 2) of h[k] a[n] + g[k] d[n],
// n = ((m - k) / 2) mod (by / 2)
template <class C>
__global__ void k_idwt_y(const C* __restrict__ in, C* __restrict__ out, int ny, int nx, int by, int bx) {
  using R = typename Real<C>::T;
  const int half = by / 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)by * bx) return;
  const int m = (int)(t / bx), x = (int)(t % bx);
  const size_t img = (size_t)blockIdx.y * ny * nx;
  C acc = czero<C>();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 2 * kk + (m & 1);
    int n = (m - k) / 2;            // m - k is even
    n = ((n % half) + half) % half;
    acc = cfma(acc, wav_h<R>(k), in[img + (size_t)n * nx + x]);
    acc = cfma(acc, wav_g<R>(k), in[img + (size_t)(half + n) * nx + x]);
  }
  out[img + (size_t)m * nx + x] = acc;
}

// synthesis along x
template <class C>
__global__ void k_idwt_x(const C* __restrict__ in, C* __restrict__ out, int ny, int nx, int by, int bx) {
  using R = typename Real<C>::T;
  const int half = bx / 2;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)by * bx) return;
  const int y = (int)(t / bx), m = (int)(t % bx);
  const size_t img = (size_t)blockIdx.y * ny * nx;
  const C* row = in + img + (size_t)y * nx;
  C acc = czero<C>();
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 2 * kk + (m & 1);
    int n = (m - k) / 2;
    n = ((n % half) + half) % half;
    acc = cfma(acc, wav_h<R>(k), row[n]);
    acc = cfma(acc, wav_g<R>(k), row[half + n]);
  }
  out[img + (size_t)y * nx + m] = acc;
}

// One analysis level of the block (by, bx) of each image with both axes in
// one pass through LDS (the layout the two one-axis passes leave: [a | d]
// along x, then along y).  A workgroup takes 16 x 16 positions of each
// subband from input rows / cols 2 j0 .. 2 j0 + 37 (periodic in the block),
// so the level reads and writes the block once.  The input block starts at
// row ri of `in`; the details go to their final places in `out`, the
// low-low subband to `ll` from row rl (the next level's input, or its final
// place at the last level).  DSOFT: the soft-threshold derivative at ck is
// applied to the details as they are written.  GRAD: the input is the FISTA
// gradient point y - (q - g) / s^2 of three fields (in = y), formed as the
// tile is loaded.
constexpr int kWT = 16, kWIn = 2 * kWT + 6;
// v mod n (n > 0), a compare and an add when v is within one period of
// [0, n) (every index of a tile whose block is at least the tile's span)
__device__ __forceinline__ int wrapmod(int v, int n) {
  if (v >= 0 && v < n) return v;
  if (v < 0 && v >= -n) return v + n;
  if (v >= n && v < 2 * n) return v - n;
  return ((v % n) + n) % n;
}
template <class C, bool DSOFT, bool GRAD>
__global__ __launch_bounds__(256) void k_dwt2(const C* __restrict__ in, int ri, C* __restrict__ out,
                                              C* __restrict__ ll, int rl, int ny, int nx, int by, int bx,
                                              const double2* __restrict__ ck, double lam, const C* __restrict__ q,
                                              const C* __restrict__ gr, float inv_s2) {
  using R = typename Real<C>::T;
  __shared__ C sT[kWIn][kWIn + 1];     // input tile
  __shared__ C sX[kWIn][2 * kWT + 1];  // after the x pass: [a | d], 16 each
  const int hy = by / 2, hx = bx / 2;
  const int tilesx = (hx + kWT - 1) / kWT;
  const int j0 = (int)(blockIdx.x / tilesx) * kWT, i0 = (int)(blockIdx.x % tilesx) * kWT;
  const size_t img = (size_t)blockIdx.y * ny * nx;
  const int t = threadIdx.x;
  for (int e = t; e < kWIn * kWIn; e += 256) {
    const int a = e / kWIn, b = e % kWIn;
    const size_t o = img + (size_t)(ri + wrapmod(2 * j0 + a, by)) * nx + wrapmod(2 * i0 + b, bx);
    if constexpr (GRAD) sT[a][b] = cfma(in[o], -inv_s2, csub(q[o], gr[o]));
    else sT[a][b] = in[o];
  }
  __syncthreads();
  for (int e = t; e < kWIn * kWT; e += 256) {
    const int a = e / kWT, i = e % kWT;
    C lo = czero<C>(), hi = czero<C>();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const C v = sT[a][2 * i + k];
      lo = cfma(lo, wav_h<R>(k), v);
      hi = cfma(hi, wav_g<R>(k), v);
    }
    sX[a][i] = lo;
    sX[a][kWT + i] = hi;
  }
  __syncthreads();
  for (int e = t; e < 2 * kWT * kWT; e += 256) {
    const int j = e / (2 * kWT), c = e % (2 * kWT);   // c < 16: x-low column i = c, else x-high
    C lo = czero<C>(), hi = czero<C>();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const C v = sX[2 * j + k][c];
      lo = cfma(lo, wav_h<R>(k), v);
      hi = cfma(hi, wav_g<R>(k), v);
    }
    const int gj = j0 + j, gi = i0 + c % kWT;
    if (gj < hy && gi < hx) {
      if (c < kWT) {
        ll[img + (size_t)(rl + gj) * nx + gi] = lo;
      } else {
        const size_t ilo = (size_t)gj * nx + hx + gi;
        if constexpr (DSOFT) lo = dsoft_one(lo, ck[ilo], lam);
        out[img + ilo] = lo;
      }
      const size_t ihi = (size_t)(hy + gj) * nx + (c < kWT ? 0 : hx) + gi;
      if constexpr (DSOFT) hi = dsoft_one(hi, ck[ihi], lam);
      out[img + ihi] = hi;
    }
  }
}

// One synthesis level of the block (by, bx) with both axes in one pass, out
// of place: 32 x 32 output points per workgroup from 20 x 20 windows of the
// four subbands (coefficient rows / cols m0 / 2 - 4 .. m0 / 2 + 15, periodic
// in the half block), y synthesis into LDS, then x synthesis.  The details
// come from `in`, the low-low subband from `llb` from row rl; the block is
// written to `out` from row ro.  MOM: FISTA momentum on the image.
constexpr int kST = 32, kSW = kST / 2 + 4;
__device__ __forceinline__ int pmod(int v, int n) { return wrapmod(v, n); }
template <class C, bool MOM>
__global__ __launch_bounds__(256) void k_idwt2(const C* __restrict__ in, const C* __restrict__ llb, int rl,
                                               C* __restrict__ out, int ro, int ny, int nx, int by, int bx,
                                               C* __restrict__ y, float theta) {
  using R = typename Real<C>::T;
  __shared__ C sC[2 * kSW][2 * kSW + 1];   // [y-low | y-high] x [x-low | x-high] windows
  __shared__ C sY[kST][2 * kSW + 1];       // after the y synthesis: 32 rows x [x-low | x-high]
  const int hy = by / 2, hx = bx / 2;
  const int tilesx = (bx + kST - 1) / kST;
  const int m0 = (int)(blockIdx.x / tilesx) * kST, c0 = (int)(blockIdx.x % tilesx) * kST;
  const int wy = m0 / 2 - 4, wx = c0 / 2 - 4;   // window starts (periodic)
  const size_t img = (size_t)blockIdx.y * ny * nx;
  const int t = threadIdx.x;
  // every load of the windows is issued before the first LDS store
  constexpr int NW = 4 * kSW * kSW, NIT = (NW + 255) / 256;
  C wv[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = t + 256 * it;
    if (e < NW) {
      const int a = e / (2 * kSW), b = e % (2 * kSW);
      const bool lly = a < kSW, llx = b < kSW;
      const int ry = lly ? pmod(wy + a, hy) : hy + pmod(wy + a - kSW, hy);
      const int rx = llx ? pmod(wx + b, hx) : hx + pmod(wx + b - kSW, hx);
      wv[it] = (lly && llx) ? llb[img + (size_t)(rl + ry) * nx + rx] : in[img + (size_t)ry * nx + rx];
    }
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = t + 256 * it;
    if (e < NW) sC[e / (2 * kSW)][e % (2 * kSW)] = wv[it];
  }
  __syncthreads();
  // x[m] = sum over taps k = m (mod 2) of h[k] a[n] + g[k] d[n], n = (m - k) / 2
  for (int e = t; e < kST * 2 * kSW; e += 256) {
    const int mm = e / (2 * kSW), b = e % (2 * kSW), m = m0 + mm;
    C acc = czero<C>();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 2 * kk + (m & 1);
      const int ln = (m - k) / 2 - wy;   // 1 .. 19
      acc = cfma(acc, wav_h<R>(k), sC[ln][b]);
      acc = cfma(acc, wav_g<R>(k), sC[kSW + ln][b]);
    }
    sY[mm][b] = acc;
  }
  __syncthreads();
  for (int e = t; e < kST * kST; e += 256) {
    const int mm = e / kST, cc = e % kST, c = c0 + cc;
    C acc = czero<C>();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 2 * kk + (c & 1);
      const int ln = (c - k) / 2 - wx;
      acc = cfma(acc, wav_h<R>(k), sY[mm][ln]);
      acc = cfma(acc, wav_g<R>(k), sY[mm][kSW + ln]);
    }
    if (m0 + mm < by && c < bx) {
      const size_t o = img + (size_t)(ro + m0 + mm) * nx + c;
      if constexpr (MOM) {   // FISTA momentum on the image: y = x + theta (x - x_prev), x_prev = x (in out)
        const C xo = out[o];
        y[o] = cfma(acc, theta, csub(acc, xo));
      }
      out[o] = acc;
    }
  }
}

// Psi (forward) or Psi^H (inverse) of K images in place in buf, tmp as scratch
// levels l0 .. levels - 1 only (the block of level l is (ny >> l) x (nx >> l))
template <class C>
static hipError_t wavelet_levels(C* buf, C* tmp, int K, int ny, int nx, int l0, int levels, bool inverse,
                                 hipStream_t s) {
  auto grid_for = [&](long work) { return dim3((unsigned)((work + 255) / 256), K); };
  if (!inverse) {
    for (int l = l0; l < levels; ++l) {
      const int by = ny >> l, bx = nx >> l;
      hipLaunchKernelGGL(k_dwt_x<C>, grid_for((long)by * (bx / 2)), dim3(256), 0, s, buf, tmp, ny, nx, by, bx);
      hipLaunchKernelGGL(k_dwt_y<C>, grid_for((long)(by / 2) * bx), dim3(256), 0, s, tmp, buf, ny, nx, by, bx);
    }
  } else {
    for (int l = levels - 1; l >= l0; --l) {
      const int by = ny >> l, bx = nx >> l;
      hipLaunchKernelGGL(k_idwt_y<C>, grid_for((long)by * bx), dim3(256), 0, s, buf, tmp, ny, nx, by, bx);
      hipLaunchKernelGGL(k_idwt_x<C>, grid_for((long)by * bx), dim3(256), 0, s, tmp, buf, ny, nx, by, bx);
    }
  }
  return hipGetLastError();
}

template <class C>
static hipError_t wavelet(C* buf, C* tmp, int K, int ny, int nx, int levels, bool inverse, hipStream_t s) {
  return wavelet_levels(buf, tmp, K, ny, nx, 0, levels, inverse, s);
}

static dim3 grid1(long n, int K = 1) { return dim3((unsigned)((n + 255) / 256), K); }

__device__ __forceinline__ bool is_detail(long i, int nx, int ly, int lx) {
  const int y = (int)(i / nx), x = (int)(i % nx);
  return !(y < ly && x < lx);
}

// z = y - (q - g) * inv_s2 over K images; g has K images or one shared (gK = 0)
__global__ void k_fista_grad(const float2* __restrict__ y, const float2* __restrict__ q,
                             const float2* __restrict__ g, float2* __restrict__ z, long n, int gK,
                             float inv_s2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)k * n + i;
  const float2 gv = g[(gK ? (size_t)k * n : 0) + i];
  z[o] = cfma(y[o], -inv_s2, csub(q[o], gv));
}

// y = xn + theta (xn - xo); xo = xn   (K images)
__global__ void k_momentum(const float2* __restrict__ xn, float2* __restrict__ xo, float2* __restrict__ y,
                           long total, float theta) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const float2 a = xn[i], b = xo[i];
  y[i] = cfma(a, theta, csub(a, b));
  xo[i] = a;
}

// sum += |u|^2, sumsq += |u|^4 over the K tangent images, in probe order
__global__ void k_accum_abs2(const float2* __restrict__ u, double* __restrict__ sum,
                             double* __restrict__ sum_im, double* __restrict__ sumsq, int K, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, si = 0.0, ss = 0.0;
  for (int k = 0; k < K; ++k) {
    const float2 v = u[(size_t)k * n + i];
    const double p = (double)v.x * v.x + (double)v.y * v.y;
    s += p;
    si += (double)v.x;
    ss += p * p;
  }
  sum[i] += s;
  if (sum_im) sum_im[i] += si;
  if (sumsq) sumsq[i] += ss;
}

__global__ void k_fill_zero(float2* __restrict__ a, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) a[i] = make_float2(0.f, 0.f);
}


hipError_t launch_fista_grad(const float2* y, const float2* q, const float2* g, float2* z, long n, int K,
                             int gK, float inv_s2, hipStream_t s) {
  hipLaunchKernelGGL(k_fista_grad, grid1(n, K), dim3(256), 0, s, y, q, g, z, n, gK, inv_s2);
  return hipGetLastError();
}

// Tangent analysis of the gradient point z = y - (q - g) * inv_s2 (K images
// each) into coefficients in dst, the soft-threshold derivative at ck applied
// to every detail coefficient as it is written.  Each level is one fused
// pass; level l (block by = ny >> l) reads its input block from scratch rows
// [by, 2 by) (level 0: z, formed as the tiles load) and writes its low-low
// subband to scratch rows [by / 2, by), disjoint from its input (the last
// level: to its final place in dst).
hipError_t launch_cs_analysis(const float2* y, const float2* q, const float2* g, float inv_s2, float2* scratch,
                              float2* dst, int K, int ny, int nx, int levels, const double2* ck, double lam,
                              hipStream_t s) {
  if (levels < 1) return hipErrorInvalidValue;
  const bool ds = lam != 0.0;
  for (int l = 0; l < levels; ++l) {
    const int by = ny >> l, bx = nx >> l;
    const dim3 grid((unsigned)(((by / 2 + kWT - 1) / kWT) * ((bx / 2 + kWT - 1) / kWT)), (unsigned)K);
    const bool last = l == levels - 1;
    float2* ll = last ? dst : scratch;
    const int rl = last ? 0 : by / 2;
    if (l == 0) {
      if (ds) hipLaunchKernelGGL((k_dwt2<float2, true, true>), grid, dim3(256), 0, s, y, 0, dst, ll, rl, ny, nx, by,
                                 bx, ck, lam, q, g, inv_s2);
      else hipLaunchKernelGGL((k_dwt2<float2, false, true>), grid, dim3(256), 0, s, y, 0, dst, ll, rl, ny, nx, by,
                              bx, ck, lam, q, g, inv_s2);
    } else {
      const float2* in = scratch;
      if (ds) hipLaunchKernelGGL((k_dwt2<float2, true, false>), grid, dim3(256), 0, s, in, by, dst, ll, rl, ny, nx,
                                 by, bx, ck, lam, q, g, inv_s2);
      else hipLaunchKernelGGL((k_dwt2<float2, false, false>), grid, dim3(256), 0, s, in, by, dst, ll, rl, ny, nx,
                              by, bx, ck, lam, q, g, inv_s2);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Tangent synthesis of the coefficients in src (read only) with the FISTA
// momentum: the image x replaces x_prev in xo and y = x + theta (x - x_prev).
// Each level is one fused pass; level l (block by = ny >> l) takes its
// low-low subband from scratch rows [by / 2, by) (the coarsest level: from
// src) and writes its block to scratch rows [by, 2 by), disjoint from that
// input (level 0: the image, into xo with the momentum).
hipError_t launch_cs_synthesis(const float2* src, float2* scratch, int K, int ny, int nx, int levels, float2* xo,
                               float2* y, float theta, hipStream_t s) {
  if (levels < 1) return hipErrorInvalidValue;
  for (int l = levels - 1; l >= 0; --l) {
    const int by = ny >> l, bx = nx >> l;
    const dim3 grid((unsigned)(((by + kST - 1) / kST) * ((bx + kST - 1) / kST)), (unsigned)K);
    const float2* llb = l == levels - 1 ? src : scratch;
    const int rl = l == levels - 1 ? 0 : by / 2;
    if (l == 0)
      hipLaunchKernelGGL((k_idwt2<float2, true>), grid, dim3(256), 0, s, src, llb, rl, xo, 0, ny, nx, by, bx, y,
                         theta);
    else
      hipLaunchKernelGGL((k_idwt2<float2, false>), grid, dim3(256), 0, s, src, llb, rl, scratch, by, ny, nx, by, bx,
                         y, theta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_momentum(const float2* xn, float2* xo, float2* y, long total, float theta,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_momentum, grid1(total), dim3(256), 0, s, xn, xo, y, total, theta);
  return hipGetLastError();
}

hipError_t launch_accum_abs2(const float2* u, double* sum, double* sum_im, double* sumsq, int K, long n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_accum_abs2, grid1(n), dim3(256), 0, s, u, sum, sum_im, sumsq, K, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float2* a, long total, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, grid1(total), dim3(256), 0, s, a, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 linearisation point.  The Jacobian is evaluated at the reconstruction's
// own trajectory, and the soft-threshold active sets (|c| > lam) decide the
// tangent map; an FP32 trajectory flips coefficients lying within its rounding
// of the threshold, so the primal (power method, FISTA, stored c_k) runs in
// FP64, once per operator.  The normal operator uses the centred orthonormal
// DFT as dense matrix products: F[k][n] = exp(-2 pi i (k - N/2)(n - N/2) / N) / sqrt(N),
// symmetric, so A_c y = F_y (S_c y) F_x and A_c^H z = conj(F_y) z conj(F_x).

__global__ void k_centred_dft64(double2* __restrict__ F, int N) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * N) return;
  const long k = i / N - N / 2, m = i % N - N / 2;
  long p = (k * m) % N;
  if (p < 0) p += N;
  double s, c;
  sincospi(-2.0 * (double)p / (double)N, &s, &c);
  const double r = 1.0 / sqrt((double)N);
  F[i] = make_double2(c * r, s * r);
}

// S[c] = sum_{d <= c} Linv[c][d] maps[d]   (whitened coil maps, centred order)
__global__ void k_prep_maps64(const float2* __restrict__ maps, const double* __restrict__ linv,
                              double2* __restrict__ S, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < nc; ++c) {
    double re = 0.0, im = 0.0;
    for (int d = 0; d <= c; ++d) {
      const double lr = linv[2 * (c * nc + d)], li = linv[2 * (c * nc + d) + 1];
      const float2 m = maps[(size_t)d * n + i];
      re += lr * m.x - li * m.y;
      im += lr * m.y + li * m.x;
    }
    S[(size_t)c * n + i] = make_double2(re, im);
  }
}

// U[c] = mask * sum_{d <= c} Linv[c][d] kdata[d]   (whitened, sampled k-space)
__global__ void k_whiten64(const float2* __restrict__ kd, const double* __restrict__ linv,
                           const uint8_t* __restrict__ mask, double2* __restrict__ U, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool on = mask[i] != 0;
  for (int c = 0; c < nc; ++c) {
    double re = 0.0, im = 0.0;
    for (int d = 0; on && d <= c; ++d) {
      const double lr = linv[2 * (c * nc + d)], li = linv[2 * (c * nc + d) + 1];
      const float2 m = kd[(size_t)d * n + i];
      re += lr * m.x - li * m.y;
      im += lr * m.y + li * m.x;
    }
    U[(size_t)c * n + i] = make_double2(re, im);
  }
}

// U[b][c] = S_c y[b]   (batch b = blockIdx.y)
__global__ void k_mul_maps64(const double2* __restrict__ y, const double2* __restrict__ S,
                             double2* __restrict__ U, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  const double2 v = y[(size_t)b * n + i];
  double2* Ub = U + (size_t)b * nc * n;
  for (int c = 0; c < nc; ++c) {
    const double2 m = S[(size_t)c * n + i];
    Ub[(size_t)c * n + i] = make_double2(m.x * v.x - m.y * v.y, m.x * v.y + m.y * v.x);
  }
}

// U[b][c][i] = mask[i] sigma n, n a CN(0, 1) Philox draw (stream 1, element
// c n + i, draw first + b): the PMR perturbation of whitened k-space
__global__ void k_noise64(double2* __restrict__ U, const uint8_t* __restrict__ mask, int nc, long n,
                          uint64_t seed, uint64_t first, double sigma) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  for (int c = 0; c < nc; ++c) {
    double2 v = make_double2(0.0, 0.0);
    if (mask[i]) {
      const float2 d = draw_probe(seed, first + b, (uint32_t)((size_t)c * n + i), 1u, 3);
      v = make_double2(sigma * (double)d.x, sigma * (double)d.y);
    }
    U[((size_t)b * nc + c) * n + i] = v;
  }
}

// out[b][i] += base[i]
__global__ void k_add_bcast64(double2* __restrict__ out, const double2* __restrict__ base, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  double2& o = out[(size_t)b * n + i];
  o = make_double2(o.x + base[i].x, o.y + base[i].y);
}

// d = (x[b] - x0) / sigma over the B replicas in order: sum Re d, sum Im d, sum |d|^2
__global__ void k_accum_pmr64(const double2* __restrict__ x, const double2* __restrict__ x0, double inv_sigma,
                              double* __restrict__ sum, double* __restrict__ sum_im, double* __restrict__ sumsq,
                              int B, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0, si = 0.0, ss = 0.0;
  for (int b = 0; b < B; ++b) {
    const double2 v = x[(size_t)b * n + i];
    const double dr = (v.x - x0[i].x) * inv_sigma, di = (v.y - x0[i].y) * inv_sigma;
    s += dr;
    si += di;
    ss += dr * dr + di * di;
  }
  sum[i] += s;
  sum_im[i] += si;
  sumsq[i] += ss;
}

__global__ void k_mask64(double2* __restrict__ U, const uint8_t* __restrict__ mask, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || mask[i]) return;
  for (int c = 0; c < nc; ++c) U[(size_t)c * n + i] = make_double2(0.0, 0.0);
}

// out[b] = sum_c conj(S_c) U[b][c]   (batch b = blockIdx.y)
__global__ void k_combine64(const double2* __restrict__ U, const double2* __restrict__ S,
                            double2* __restrict__ out, int nc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  const double2* Ub = U + (size_t)b * nc * n;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double2 m = S[(size_t)c * n + i], u = Ub[(size_t)c * n + i];
    re += m.x * u.x + m.y * u.y;
    im += m.x * u.y - m.y * u.x;
  }
  out[(size_t)b * n + i] = make_double2(re, im);
}

// unit random-phase start of the power method (Philox stream 3, key 0, draw 0)
__global__ void k_power_start64(double2* __restrict__ v, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const u32x4 w = philox4x32_10((uint32_t)i, 0u, 0u, 3u, 0u, 0u);
  double s, c;
  sincospi((double)(w.w0 >> 8) * 0x1p-23, &s, &c);   // 2 pi f, f = (w0 >> 8) / 2^24
  const double r = 1.0 / sqrt((double)n);
  v[i] = make_double2(c * r, s * r);
}

// per-block partials (Re v^H w, |w|^2), fixed reduction order
__global__ __launch_bounds__(256) void k_dot64(const double2* __restrict__ v, const double2* __restrict__ w,
                                               double* __restrict__ part, long n) {
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double2 x = v[i], y = w[i];
    a += x.x * y.x + x.y * y.y;
    b += y.x * y.x + y.y * y.y;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

__global__ void k_scale64(const double2* __restrict__ w, double2* __restrict__ v, long n, double sc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = make_double2(w[i].x * sc, w[i].y * sc);
}

// z = y - (q - g) * inv_s2
__global__ void k_grad64(const double2* __restrict__ y, const double2* __restrict__ q,
                         const double2* __restrict__ g, double2* __restrict__ z, long n, double inv_s2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  z[i] = make_double2(y[i].x - (q[i].x - g[i].x) * inv_s2, y[i].y - (q[i].y - g[i].y) * inv_s2);
}

// c_k stored (when store is given), then detail coefficients soft-thresholded
// in place; total = B images of img pixels each
__global__ void k_soft_store64(double2* __restrict__ c, double2* __restrict__ store, long total, long img,
                               int nx, int ly, int lx, double lam) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const double2 v = c[i];
  if (store) store[i] = v;
  if (is_detail(i % img, nx, ly, lx)) {
    const double a = sqrt(v.x * v.x + v.y * v.y);
    const double sc = a > lam ? 1.0 - lam / a : 0.0;
    c[i] = make_double2(v.x * sc, v.y * sc);
  }
}

// y = xn + theta (xn - xo); xo = xn
__global__ void k_momentum64(const double2* __restrict__ xn, double2* __restrict__ xo, double2* __restrict__ y,
                             long n, double theta) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 a = xn[i], b = xo[i];
  y[i] = make_double2(fma(theta, a.x - b.x, a.x), fma(theta, a.y - b.y, a.y));
  xo[i] = a;
}

__global__ void k_to_f32(const double2* __restrict__ a, float2* __restrict__ b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void k_fill_zero64(double2* __restrict__ a, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = make_double2(0.0, 0.0);
}

#define CS_CHECK(x)            \
  do {                         \
    hipError_t e_ = (x);       \
    if (e_ != hipSuccess) return e_; \
  } while (0)

hipError_t cs64_setup(Cs64& o, const float2* maps, const double* linv, hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  hipLaunchKernelGGL(k_centred_dft64, grid1((long)o.ny * o.ny), dim3(256), 0, s, o.Fy, o.ny);
  hipLaunchKernelGGL(k_centred_dft64, grid1((long)o.nx * o.nx), dim3(256), 0, s, o.Fx, o.nx);
  hipLaunchKernelGGL(k_prep_maps64, grid1(n), dim3(256), 0, s, maps, linv, o.S, o.nc, n);
  return hipGetLastError();
}

// out[b] = sum_c conj(S_c) A_c^H of the k-space held in o.U [B][nc] (overwritten)
static hipError_t cs64_adjoint_u(const Cs64& o, int B, double2* out, hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  const int P = B * o.nc;
  CS_CHECK(zgemm64(o.Fy, o.U, o.V, o.ny, o.nx, o.ny, 2, 1, s, P, 0, n, n));     // conj(F_y) U_bc
  CS_CHECK(zgemm64(o.V, o.Fx, o.U, P * o.ny, o.nx, o.nx, 4, 1, s));              // . conj(F_x)
  hipLaunchKernelGGL(k_combine64, grid1(n, B), dim3(256), 0, s, o.U, o.S, out, o.nc, n);
  return hipGetLastError();
}

// q[b] = M y[b] for B images
hipError_t cs64_normal(const Cs64& o, int B, const double2* y, double2* q, hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  const int P = B * o.nc;
  hipLaunchKernelGGL(k_mul_maps64, grid1(n, B), dim3(256), 0, s, y, o.S, o.U, o.nc, n);
  CS_CHECK(zgemm64(o.U, o.Fx, o.V, P * o.ny, o.nx, o.nx, 0, 1, s));              // (S_c y) F_x
  CS_CHECK(zgemm64(o.Fy, o.V, o.U, o.ny, o.nx, o.ny, 0, 1, s, P, 0, n, n));     // F_y .
  hipLaunchKernelGGL(k_mask64, grid1(n), dim3(256), 0, s, o.U, o.mask, P, n);
  return cs64_adjoint_u(o, B, q, s);
}

hipError_t cs64_adjoint_kdata(const Cs64& o, const float2* kdata, const double* linv, double2* out,
                              hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  hipLaunchKernelGGL(k_whiten64, grid1(n), dim3(256), 0, s, kdata, linv, o.mask, o.U, o.nc, n);
  return cs64_adjoint_u(o, 1, out, s);
}

// lambda_max of M: power steps from the Philox start; Rayleigh quotient of the last step
hipError_t cs64_power(const Cs64& o, int iters, double2* v, double2* w, double* part_d, double* out,
                      hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  const int nb = (int)std::min<long>((n + 255) / 256, CS64_DOT_BLOCKS);
  std::vector<double> part(2 * (size_t)nb);
  hipLaunchKernelGGL(k_power_start64, grid1(n), dim3(256), 0, s, v, n);
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    CS_CHECK(cs64_normal(o, 1, v, w, s));
    hipLaunchKernelGGL(k_dot64, dim3(nb), dim3(256), 0, s, v, w, part_d, n);
    CS_CHECK(hipMemcpyAsync(part.data(), part_d, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    CS_CHECK(hipStreamSynchronize(s));
    double vw = 0.0, ww = 0.0;
    for (int b = 0; b < nb; ++b) {
      vw += part[2 * b];
      ww += part[2 * b + 1];
    }
    lam = vw;
    if (!(ww > 0.0)) break;
    hipLaunchKernelGGL(k_scale64, grid1(n), dim3(256), 0, s, w, v, n, 1.0 / sqrt(ww));
  }
  *out = lam;
  return hipGetLastError();
}

// T FISTA iterations on B images from x_0 = y_1 = 0 (atb [B][n]), leaving x_T
// in x.  With store (B = 1 only) the trajectory the tangents need is kept:
// c_k = Psi z_k in o.ctraj (wavelet prox) or the TV projection data in
// o.tv_what / o.tv_invn.  Buffers y, x, z, tmp, q hold B images each.
hipError_t cs64_fista(const Cs64& o, int B, const double2* atb, double s2, double lam, int T,
                      const double* theta, bool store, double2* y, double2* x, double2* z,
                      double2* tmp, double2* q, hipStream_t s) {
  const long n = (long)o.ny * o.nx, tot = n * B;
  const int ly = o.ny >> o.levels, lx = o.nx >> o.levels;
  hipLaunchKernelGGL(k_fill_zero64, grid1(tot), dim3(256), 0, s, y, tot);
  hipLaunchKernelGGL(k_fill_zero64, grid1(tot), dim3(256), 0, s, x, tot);
  for (int k = 1; k <= T; ++k) {
    CS_CHECK(cs64_normal(o, B, y, q, s));
    hipLaunchKernelGGL(k_grad64, grid1(tot), dim3(256), 0, s, y, q, atb, z, tot, 1.0 / s2);
    if (o.tv_inner > 0) {
      const size_t off = (size_t)(k - 1) * o.tv_inner * n;
      CS_CHECK(tv64_prox(o, B, z, lam, store ? o.tv_what + off : nullptr, store ? o.tv_invn + off : nullptr, s));
    } else {
      CS_CHECK(wavelet(z, tmp, B, o.ny, o.nx, o.levels, false, s));
      hipLaunchKernelGGL(k_soft_store64, grid1(tot), dim3(256), 0, s, z,
                         store ? o.ctraj + (size_t)(k - 1) * n : nullptr, tot, n, o.nx, ly, lx, lam);
      CS_CHECK(wavelet(z, tmp, B, o.ny, o.nx, o.levels, true, s));
    }
    hipLaunchKernelGGL(k_momentum64, grid1(tot), dim3(256), 0, s, z, x, y, tot, theta[k - 1]);
  }
  return hipGetLastError();
}

// B PMR replicas of the FP64 reconstruction: x_b = f(b_w + sigma n_b), then
// (x_b - x0) / sigma accumulated into sum, sum_im, sumsq
hipError_t cs64_pmr(const Cs64& o, int B, const double2* atb0, const double2* x0, double s2, double lam,
                    int T, const double* theta, uint64_t seed, uint64_t first, double sigma, double2* atb,
                    double2* y, double2* x, double2* z, double2* tmp, double2* q, double* sum,
                    double* sum_im, double* sumsq, hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  hipLaunchKernelGGL(k_noise64, grid1(n, B), dim3(256), 0, s, o.U, o.mask, o.nc, n, seed, first, sigma);
  CS_CHECK(cs64_adjoint_u(o, B, atb, s));                                        // A^H (sigma n_b)
  hipLaunchKernelGGL(k_add_bcast64, grid1(n, B), dim3(256), 0, s, atb, atb0, n);   // + A^H b_w
  CS_CHECK(cs64_fista(o, B, atb, s2, lam, T, theta, false, y, x, z, tmp, q, s));
  hipLaunchKernelGGL(k_accum_pmr64, grid1(n), dim3(256), 0, s, x, x0, 1.0 / sigma, sum, sum_im, sumsq, B, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double2* a, float2* b, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, grid1(n), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

}  // namespace pico
