// Construction of the Toeplitz weights for a non-Cartesian trajectory, once
// per operator, in float64:
//   psf(d) = N_x^-1 sum_m exp(i w_m . d),  d in [-(ny-1), ny-1] x [-(nx-1), nx-1],
// evaluated separably as a complex matrix product psf = E_y^T E_x with
// E_y[m][j] = exp(i w_y,m (j - ny + 1)), E_x likewise (a dense contraction
// over the M samples, taken in chunks of samples); circulant embedding in a 2ny x 2nx grid; its DFT by
// two more products with DFT matrices; W = Re(DFT) / (4 ny nx), transposed.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "runtime.h"

namespace pico {

using z64 = double2;

__global__ void k_exp_table(const float* __restrict__ traj, int comp, int d0, int D, int M,
                            z64* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)M * D) return;
  const int m = (int)(i / D), j = (int)(i % D);
  const double w = (double)traj[2 * (size_t)m + comp];
  double s, c;
  sincos(w * (double)(d0 + j), &s, &c);
  out[i] = make_double2(c, s);
}

// C[z][i][j] = sum_{kk in slice z} op(A)[i][kk] op(B)[kk][j]; op(A) = A (A: [Mr][Kd])
// or A^T (A: [Kd][Mr]), optionally conjugated; op(B) = B or conj(B), B: [Kd][Nc];
// row-major complex128; 32x32 tile per block.  flags: 1 transA, 2 conjA, 4 conjB.
// blockIdx.z = batch * S + slice; batch b offsets A, B, C by b * sA, sB, sC.
__global__ __launch_bounds__(256) void k_zgemm(const z64* __restrict__ A, const z64* __restrict__ B,
                                               z64* __restrict__ C, int Mr, int Nc, int Kd,
                                               int flags, int kslice, int S, long sA, long sB,
                                               long sC) {
  const int transA = flags & 1;
  const int bz = blockIdx.z / S, sl = blockIdx.z % S;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  __shared__ z64 As[16][33];
  __shared__ z64 Bs[16][33];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int kbeg = sl * kslice, kend = min(Kd, kbeg + kslice);
  double acc[2][2][2] = {};
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 32; e += 256) {
      const int kk = e / 32, ii = e % 32;
      const int gk = k0 + kk, gi = i0 + ii, gj = j0 + ii;
      z64 av = make_double2(0.0, 0.0), bv = make_double2(0.0, 0.0);
      if (gk < kend && gi < Mr) av = transA ? A[(size_t)gk * Mr + gi] : A[(size_t)gi * Kd + gk];
      if (gk < kend && gj < Nc) bv = B[(size_t)gk * Nc + gj];
      if (flags & 2) av.y = -av.y;
      if (flags & 4) bv.y = -bv.y;
      As[kk][ii] = av;
      Bs[kk][ii] = bv;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const z64 x = As[kk][ty + 16 * a];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const z64 y = Bs[kk][tx + 16 * b];
          acc[a][b][0] = fma(x.x, y.x, fma(-x.y, y.y, acc[a][b][0]));
          acc[a][b][1] = fma(x.x, y.y, fma(x.y, y.x, acc[a][b][1]));
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gi = i0 + ty + 16 * a, gj = j0 + tx + 16 * b;
      if (gi < Mr && gj < Nc)
        C[((size_t)sl * Mr + gi) * Nc + gj] = make_double2(acc[a][b][0], acc[a][b][1]);
    }
}

// sum over split-K slices in slice order, scaled; added to out when accumulate
__global__ void k_zsum_slices(const z64* __restrict__ parts, z64* __restrict__ out, long n, int S,
                              double scale, int accumulate) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  for (int z = 0; z < S; ++z) {
    re += parts[(size_t)z * n + i].x;
    im += parts[(size_t)z * n + i].y;
  }
  z64 v = make_double2(re * scale, im * scale);
  if (accumulate) {
    v.x += out[i].x;
    v.y += out[i].y;
  }
  out[i] = v;
}

// k[dy mod Gy][dx mod Gx] = psf[dy + ny - 1][dx + nx - 1]; zero elsewhere
__global__ void k_embed(const z64* __restrict__ psf, z64* __restrict__ kg, int ny, int nx, int Gy,
                        int Gx) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)Gy * Gx) return;
  const int ky = (int)(i / Gx), kx = (int)(i % Gx);
  const int dy = ky < ny ? ky : ky - Gy;  // index ny maps to -ny: outside the PSF support
  const int dx = kx < nx ? kx : kx - Gx;
  z64 v = make_double2(0.0, 0.0);
  if (dy > -ny && dy < ny && dx > -nx && dx < nx)
    v = psf[(size_t)(dy + ny - 1) * (2 * nx - 1) + (dx + nx - 1)];
  kg[i] = v;
}

// F[k][n] = exp(-2 pi i k n / G)
__global__ void k_dft_matrix(z64* __restrict__ F, int G) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)G * G) return;
  const long k = i / G, n = i % G;
  double s, c;
  sincospi(-2.0 * (double)((k * n) % G) / (double)G, &s, &c);
  F[i] = make_double2(c, s);
}

// w[kx][ky] = Re(Kh[ky][kx]) * scale
__global__ void k_real_weights(const z64* __restrict__ kh, float* __restrict__ w, int Gy, int Gx,
                               double scale) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)Gy * Gx) return;
  const int ky = (int)(i / Gx), kx = (int)(i % Gx);
  w[(size_t)kx * Gy + ky] = (float)(kh[i].x * scale);
}

hipError_t zgemm64(const double2* A, const double2* B, double2* C, int Mr, int Nc, int Kd,
                   int flags, int splits, hipStream_t s, int batch, long sA, long sB, long sC) {
  const int kslice = ((Kd + splits - 1) / splits + 15) / 16 * 16;
  const int S = (Kd + kslice - 1) / kslice;
  dim3 grid((Nc + 31) / 32, (Mr + 31) / 32, S * batch), block(256);
  hipLaunchKernelGGL(k_zgemm, grid, block, 0, s, A, B, C, Mr, Nc, Kd, flags, kslice, S, sA, sB, sC);
  return hipGetLastError();
}

static int zgemm_slices(int Kd, int splits) {
  const int kslice = ((Kd + splits - 1) / splits + 15) / 16 * 16;
  return (Kd + kslice - 1) / kslice;
}

// samples per chunk of the separable PSF product (bounds the exponential tables)
constexpr long kPsfChunk = 16384;
constexpr int kPsfSplits = 4;

static size_t piece(size_t count) { return (count * sizeof(z64) + 255) / 256 * 256; }

struct ToeplitzScratch {
  size_t off[9];
  size_t total;
  ToeplitzScratch(long M, int ny, int nx) {
    const long Mc = std::min<long>(M, kPsfChunk);
    const size_t Dy = 2 * ny - 1, Dx = 2 * nx - 1, Gy = 2 * ny, Gx = 2 * nx;
    const int S = zgemm_slices((int)Mc, kPsfSplits);
    const size_t sizes[9] = {piece(Mc * Dy), piece(Mc * Dx), piece((size_t)S * Dy * Dx), piece(Dy * Dx),
                             piece(Gy * Gx),  piece(Gy * Gy), piece(Gx * Gx), piece(Gy * Gx), piece(Gy * Gx)};
    total = 0;
    for (int i = 0; i < 9; ++i) {
      off[i] = total;
      total += sizes[i];
    }
  }
};

size_t toeplitz_scratch_bytes(long M, int ny, int nx) { return ToeplitzScratch(M, ny, nx).total; }

#define TZ_CHECK(x)                \
  do {                             \
    hipError_t e_ = (x);           \
    if (e_ != hipSuccess) return e_; \
  } while (0)

hipError_t build_toeplitz_weights(const float* traj, long M, int ny, int nx, float* w, void* scratch,
                                  hipStream_t s) {
  const int Dy = 2 * ny - 1, Dx = 2 * nx - 1, Gy = 2 * ny, Gx = 2 * nx;
  const ToeplitzScratch L(M, ny, nx);
  char* base = static_cast<char*>(scratch);
  z64* Ey = reinterpret_cast<z64*>(base + L.off[0]);
  z64* Ex = reinterpret_cast<z64*>(base + L.off[1]);
  z64* parts = reinterpret_cast<z64*>(base + L.off[2]);
  z64* psf = reinterpret_cast<z64*>(base + L.off[3]);
  z64* kg = reinterpret_cast<z64*>(base + L.off[4]);
  z64* Fy = reinterpret_cast<z64*>(base + L.off[5]);
  z64* Fx = reinterpret_cast<z64*>(base + L.off[6]);
  z64* t1 = reinterpret_cast<z64*>(base + L.off[7]);
  z64* kh = reinterpret_cast<z64*>(base + L.off[8]);
  const long npsf = (long)Dy * Dx;
  // psf = (1 / (ny nx)) sum over sample chunks of E_y^T E_x, chunk by chunk in order
  for (long m0 = 0; m0 < M; m0 += kPsfChunk) {
    const int Mc = (int)std::min<long>(kPsfChunk, M - m0);
    const int S = zgemm_slices(Mc, kPsfSplits);
    const float* tr = traj + 2 * m0;
    hipLaunchKernelGGL(k_exp_table, dim3((unsigned)(((long)Mc * Dy + 255) / 256)), dim3(256), 0, s, tr, 0,
                       -(ny - 1), Dy, Mc, Ey);
    hipLaunchKernelGGL(k_exp_table, dim3((unsigned)(((long)Mc * Dx + 255) / 256)), dim3(256), 0, s, tr, 1,
                       -(nx - 1), Dx, Mc, Ex);
    TZ_CHECK(hipGetLastError());
    TZ_CHECK(zgemm64(Ey, Ex, parts, Dy, Dx, Mc, 1, kPsfSplits, s));
    hipLaunchKernelGGL(k_zsum_slices, dim3((unsigned)((npsf + 255) / 256)), dim3(256), 0, s, parts, psf,
                       npsf, S, 1.0 / ((double)ny * nx), m0 > 0 ? 1 : 0);
  }
  const long ng = (long)Gy * Gx;
  hipLaunchKernelGGL(k_embed, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, psf, kg, ny, nx, Gy, Gx);
  hipLaunchKernelGGL(k_dft_matrix, dim3((unsigned)(((long)Gy * Gy + 255) / 256)), dim3(256), 0, s, Fy, Gy);
  hipLaunchKernelGGL(k_dft_matrix, dim3((unsigned)(((long)Gx * Gx + 255) / 256)), dim3(256), 0, s, Fx, Gx);
  TZ_CHECK(hipGetLastError());
  TZ_CHECK(zgemm64(Fy, kg, t1, Gy, Gx, Gy, 0, 1, s));
  TZ_CHECK(zgemm64(t1, Fx, kh, Gy, Gx, Gx, 0, 1, s));
  hipLaunchKernelGGL(k_real_weights, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, kh, w, Gy, Gx,
                     1.0 / ((double)Gy * Gx));
  TZ_CHECK(hipGetLastError());
  return hipStreamSynchronize(s);
}

}  // namespace pico
