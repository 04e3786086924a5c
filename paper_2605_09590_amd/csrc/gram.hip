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

// Wave reductions on cross-lane DPP moves (no LDS round trip): quad
// permutations [1,0,3,2] and [2,3,0,1], half-row and row mirrors, then the
// row broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows 2 and
// 3; lane 63 ends with the total, which readlane hands to every lane.  Lanes
// of rows a broadcast leaves out read 0, the identity of both reductions
// (the maximum is taken over magnitudes).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp32<CTRL, ROWS>((uint32_t)b), hi = dpp32<CTRL, ROWS>((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp64<0xb1, 0xf>(v);
  v += dpp64<0x4e, 0xf>(v);
  v += dpp64<0x141, 0xf>(v);
  v += dpp64<0x140, 0xf>(v);
  v += dpp64<0x142, 0xa>(v);
  v += dpp64<0x143, 0xc>(v);
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, lo | (hi << 32));
}
__device__ __forceinline__ float wave_max_abs(float v) {   // v >= 0 on every lane
  v = fmaxf(v, __uint_as_float(dpp32<0xb1, 0xf>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp32<0x4e, 0xf>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp32<0x141, 0xf>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp32<0x140, 0xf>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp32<0x142, 0xa>(__float_as_uint(v))));
  v = fmaxf(v, __uint_as_float(dpp32<0x143, 0xc>(__float_as_uint(v))));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Element (row, probe) of the p / q tile: rows of 32 float2 (256 B), the
// probe index XOR-swizzled by the row so that both the column writes of the
// prologue and the row reads of the matrix loop spread over the LDS banks.
__device__ __forceinline__ int tile_at(int row, int j) { return row * kTile + (j ^ (row & 31)); }

// The fused CG update in front of the product for one probe k of the tile
// (rows y = lane + 64 m, m < NM): writes x, r, p as the mode requires,
// returns p (the tile values) and adds |r|^2 to d0.  Every load of the
// column is issued before the first store, so a wave keeps the whole column
// in flight.  Inactive probes (k >= K) give zeros.
template <int MODE, int NM>
__device__ __forceinline__ void probe_column(const Cart1dArgs& a, int k, bool active, size_t base, int col, int lane,
                                             float alpha, float beta, float2 (&pv)[NM], double& d0) {
  const int ny = a.ny;
  float2 po[NM], qo[NM], ro[NM], xo[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int y = lane + 64 * m;
    pv[m] = po[m] = qo[m] = ro[m] = xo[m] = make_float2(0.f, 0.f);
    if (!active || y >= ny) continue;
    if constexpr (MODE == C1_ITER) {
      po[m] = a.p[base + y];
      qo[m] = a.q[base + y];
      ro[m] = a.r[base + y];
      if (!a.x_zero) xo[m] = a.x[base + y];
    } else if constexpr (MODE == C1_FIRST_BUF) {
      ro[m] = a.r[base + y];
    } else if constexpr (MODE == C1_APPLY) {
      pv[m] = cscale(a.src[base + y], a.scale);
    }
  }
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int y = lane + 64 * m;
    if (!active || y >= ny) continue;
    float2 rv = ro[m];
    if constexpr (MODE == C1_ITER) {
      rv = cfma(ro[m], -alpha, qo[m]);
      pv[m] = cfma(rv, beta, po[m]);
      a.x[base + y] = cfma(xo[m], alpha, po[m]);
      a.r[base + y] = rv;
      a.p[base + y] = pv[m];
    } else if constexpr (MODE == C1_FIRST_PROBE) {
      pv[m] = draw_probe(arg_seed(a), arg_first(a) + k, (uint32_t)(y * a.nx + col), 0u, a.dist);
      rv = pv[m];
      a.r[base + y] = rv;
      a.p[base + y] = rv;
    } else if constexpr (MODE == C1_FIRST_BUF) {
      pv[m] = rv;
      a.p[base + y] = rv;
    } else {
      rv = make_float2(0.f, 0.f);
    }
    d0 += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
}

// Behind the product, with q = (M_x + lam) p in the tile (tile_at layout) and
// this lane's (Re p^H q, |q|^2) partials over the wave's rows for probe li:
// store q, the Re r^H q partial per probe, then the per-probe sums of the
// other two over the waves.
template <int MODE, int NM>
__device__ __forceinline__ void gram_finish(const Cart1dArgs& a, float2* pt, int k0, int col, int w, int nw, int lane,
                                            double d1, double d2) {
  const int ny = a.ny, li = lane % 32, kk = lane / 32;
  for (int j = w; j < kTile; j += nw) {
    const int k = k0 + j;
    if (k >= a.K) continue;
    const size_t base = ((size_t)k * a.nx + col) * ny;
    float2 rv[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {   // the column of r in flight before the q stores (rows past
      const int y = min(lane + 64 * m, ny - 1);   // ny re-read the last row: no branches)
      rv[m] = MODE != C1_APPLY ? a.r[base + y] : make_float2(0.f, 0.f);
    }
    double d3 = 0.0;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const int y = lane + 64 * m;
      if (y >= ny) continue;
      const float2 q = pt[tile_at(y, j)];
      a.q[base + y] = q;
      d3 += (double)rv[m].x * q.x + (double)rv[m].y * q.y;
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
  constexpr int kRowsPerLane = SMALL ? 5 : 8;      // rows y = lane + 64 m of a column (ny <= 320 / 512)

  // ---- prologue: wave w prepares probes j = w, w + nw, ... (column-coalesced)
  for (int j = w; j < kTile; j += nw) {
    const int k = k0 + j;
    const bool active = k < a.K;
    const size_t base = ((size_t)(active ? k : 0) * a.nx + col) * ny;
    const float alpha = (MODE == C1_ITER && active) ? (float)a.alpha[k] : 0.f;
    const float beta = (MODE == C1_ITER && active) ? (float)a.beta[k] : 0.f;
    double d0 = 0.0;
    float2 pv[kRowsPerLane];
    probe_column<MODE>(a, k, active, base, col, lane, alpha, beta, pv, d0);
#pragma unroll
    for (int m = 0; m < kRowsPerLane; ++m)
      if (lane + 64 * m < ny) pt[tile_at(lane + 64 * m, j)] = pv[m];
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

  gram_finish<MODE, kRowsPerLane>(a, pt, k0, col, w, nw, lane, d1, d2);
}

// ---------------------------------------------------------------------------
// Split-FP16 form: the same blocks and CG fusion, the product on the FP16
// matrix cores (v_mfma_f32_32x32x16_f16).  Every FP32 operand a is split into
// two FP16 parts, a_hi = fl16(a) and a_lo = fl16(a - a_hi), and
//     a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// with FP32 accumulation (Ootomo and Yokota, IJHPCA 2022, "Recovering single
// precision accuracy from Tensor Cores while surpassing the FP32 theoretical
// peak performance").  The split keeps 22 of FP32's 24 significand bits and
// the dropped a_lo b_lo is below 2^-22 |a b|: per product about 2.4 times the
// error of an FP32 product.  Both operands are scaled by powers of two
// (exact) so that their largest magnitude lies in [2^14, 2^15): the block of a column by its
// largest diagonal entry (M_x is Hermitian positive semidefinite, so
// |M_x[i][j]| <= max_i M_x[i][i]), each probe of the tile by its largest
// component.  No part then overflows, and the low parts stay normal FP16
// down to ~2^-16 of the largest value, so the error stays relative to the
// largest operand rather than growing for small entries.
//
// The block of column x is stored pre-split in the operand order of the
// matrix instruction: for row block w (32 rows i), k step s (8 columns j) and
// lane l (i = 32 w + l % 32, j = 8 s + 4 (l / 32) + t, t = 0..3), four words
// (Re M_x[i][j], -Im M_x[i][j]) as packed FP16 pairs (first in the low
// half): the hi words, then the lo words, each 64 lanes x 16 bytes, so every
// load of the loop is one contiguous kilobyte.  The Im row of the product
// takes (Im, Re) = the words with halves swapped and the new low half
// negated, formed in registers.  The probe tile sits in LDS as [32][ny] hi
// words then [32][ny] lo words, 16-byte chunks XOR-swizzled by the probe.

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef uint32_t word4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_h2(_Float16 re, _Float16 im) {
  return (uint32_t)__builtin_bit_cast(uint16_t, re) | ((uint32_t)__builtin_bit_cast(uint16_t, im) << 16);
}
__device__ __forceinline__ float2 unpack_h2(uint32_t w) {
  return make_float2((float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)),
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)));
}
// (re, im) -> (-im, re): the Im-row operand from the Re-row operand
__device__ __forceinline__ word4 swap_neg(word4 v) {
  word4 o;
#pragma unroll
  for (int t = 0; t < 4; ++t) o[t] = ((v[t] >> 16) | (v[t] << 16)) ^ 0x8000u;
  return o;
}
__device__ __forceinline__ floatx16 mfma16(word4 a, word4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0, 0, 0);
}
// word index of probe j, row y in one half ([32][ny]) of the split tile
__device__ __forceinline__ int btile_at(int j, int y, int ny, int sw) {
  return j * ny + ((((y >> 2) ^ (j & sw))) << 2) + (y & 3);
}

// Block scale exponent of column x: 15 - e, max_i M_x[i][i] = f 2^e, f in [0.5, 1)
__global__ void k_gram16_scale(const float2* __restrict__ maps, const double2* __restrict__ cvec, int* __restrict__ gexp,
                               int nc, int ny) {
  __shared__ double red[256];
  const int col = blockIdx.x;
  const float2* S = maps + (size_t)col * nc * ny;
  double mx = 0.0;
  for (int i = threadIdx.x; i < ny; i += blockDim.x) {
    double d = 0.0;
    for (int c = 0; c < nc; ++c) {
      const float2 a = S[(size_t)c * ny + i];
      d += (double)a.x * a.x + (double)a.y * a.y;
    }
    mx = fmax(mx, d * cvec[0].x);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    const double m = red[0];
    if (m > 0.0 && m < INFINITY) frexp(m, &e);
    gexp[col] = 15 - e;
  }
}

// One thread per (row block, k step, lane) of a column: four entries of
// conj(M_x) in FP64, scaled, split and stored in the operand order
__global__ void k_gram16_build(const float2* __restrict__ maps, const double2* __restrict__ cvec,
                               const int* __restrict__ gexp, word4* __restrict__ G16, int nc, int ny) {
  const int nst = ny / 8;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (t >= (ny / 32) * nst * 64) return;
  const int lane = t % 64, st = (t / 64) % nst, w = t / (64 * nst);
  const int i = 32 * w + lane % 32, jb = 8 * st + 4 * (lane / 32);
  const float2* S = maps + (size_t)col * nc * ny;
  const int ge = gexp[col];
  word4 hi, lo;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = jb + u;
    double re = 0.0, im = 0.0;   // sum_c conj(S_c[i]) S_c[j]
    for (int c = 0; c < nc; ++c) {
      const float2 a = S[(size_t)c * ny + i], b = S[(size_t)c * ny + j];
      re += (double)a.x * b.x + (double)a.y * b.y;
      im += (double)a.x * b.y - (double)a.y * b.x;
    }
    const double2 cv = cvec[((i - j) % ny + ny) % ny];
    const double mr = ldexp(cv.x * re - cv.y * im, ge), mi = ldexp(cv.x * im + cv.y * re, ge);
    // operand pair (Re, -Im) of M_x[i][j]: the product row i is sum_j M[i][j] p[j]
    const _Float16 hr = (_Float16)(float)mr, hm = (_Float16)(float)(-mi);
    const _Float16 lr = (_Float16)(float)(mr - (double)(float)hr), lm = (_Float16)(float)(-mi - (double)(float)hm);
    hi[u] = pack_h2(hr, hm);
    lo[u] = pack_h2(lr, lm);
  }
  word4* o = G16 + (((size_t)col * (ny / 32) + w) * nst + st) * 128 + lane;
  o[0] = hi;
  o[64] = lo;
}

// One probe column j of the tile ahead of the product: the CG update as in the
// FP32 form, the probe's scale exponent (to pe[j]) and its split into the
// tile bt ([32][ny] hi words, then [32][ny] lo words).
template <int MODE, int NM>
__device__ __forceinline__ void split_column(const Cart1dArgs& a, uint32_t* bt, int* pe, int j, int k0, int col,
                                             int lane, int sw) {
  const int ny = a.ny, k = k0 + j;
  const bool active = k < a.K;
  const size_t base = ((size_t)(active ? k : 0) * a.nx + col) * ny;
  const float alpha = (MODE == C1_ITER && active) ? (float)a.alpha[k] : 0.f;
  const float beta = (MODE == C1_ITER && active) ? (float)a.beta[k] : 0.f;
  double d0 = 0.0;
  float2 pv[NM];
  probe_column<MODE>(a, k, active, base, col, lane, alpha, beta, pv, d0);
  float mx = 0.f;
#pragma unroll
  for (int m = 0; m < NM; ++m) mx = fmaxf(mx, fmaxf(fabsf(pv[m].x), fabsf(pv[m].y)));
  mx = wave_max_abs(mx);
  int e = 0;
  if (mx > 0.f && mx < INFINITY) frexpf(mx, &e);
  const int sp = 15 - e;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int y = lane + 64 * m;
    if (y < ny) {
      const float xr = ldexpf(pv[m].x, sp), xi = ldexpf(pv[m].y, sp);
      const _Float16 hr = (_Float16)xr, hm = (_Float16)xi;
      const int at = btile_at(j, y, ny, sw);
      bt[at] = pack_h2(hr, hm);
      bt[kTile * ny + at] = pack_h2((_Float16)(xr - (float)hr), (_Float16)(xi - (float)hm));
    }
  }
  d0 = wave_sum(d0);
  if (lane == 0) {
    pe[j] = sp;
    if (active) a.part[((size_t)k * a.nx + col) * 4] = d0;
  }
}

// The product on the matrix cores for rows [32 w, 32 w + 32) x 32 probes of
// the split tile bt, three partial products per k step (8 columns j).
__device__ __forceinline__ void tile_product(const uint32_t* bt, const word4* __restrict__ G16, int col, int w, int nw,
                                             int ny, int lane, int sw, floatx16& accR, floatx16& accI) {
  const int nst = ny / 8, li = lane % 32, kk = lane / 32, bsw = li & sw;
  const uint32_t* brow = bt + li * ny;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    accR[v] = 0.f;
    accI[v] = 0.f;
  }
  // k steps in pairs: the block words of step s + 2 load into the registers
  // step s has just used.  Buffer loads over the wave's slice of the block
  // (index clamped, so they are unconditional): as intrinsic calls they stay
  // where they are written, where plain loads feeding the loop-carried
  // registers get merged into one load at the top of the loop.
  const __amdgpu_buffer_rsrc_t gr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(G16 + (size_t)(col * nw + __builtin_amdgcn_readfirstlane(w)) * nst * 128), (short)0, nst * 2048,
      0x00020000);
  auto gload = [&](int st, int half) {
    return __builtin_amdgcn_raw_buffer_load_b128(gr, (st * 128 + half * 64 + lane) * 16, 0, 0);
  };
  auto bload = [&](int st, int half) {   // this lane's probe words of k step st
    return *reinterpret_cast<const word4*>(brow + half * kTile * ny + (((2 * st + kk) ^ bsw) << 2));
  };
  auto kstep = [&](const word4 ah, const word4 al, const word4 bh, const word4 bl) {
    accR = mfma16(ah, bh, accR);
    accR = mfma16(ah, bl, accR);
    accR = mfma16(al, bh, accR);
    const word4 aih = swap_neg(ah), ail = swap_neg(al);
    accI = mfma16(aih, bh, accI);
    accI = mfma16(aih, bl, accI);
    accI = mfma16(ail, bh, accI);
  };
  // issued in the order the loop consumes them, as the loop's own loads are,
  // so that the counter wait at the loop head covers only the first pair
  word4 h0 = gload(0, 0), l0 = gload(0, 1);
  __builtin_amdgcn_sched_barrier(0);
  word4 h1 = gload(1, 0), l1 = gload(1, 1);
  for (int st = 0; st < nst; st += 2) {
    const int n0 = min(st + 2, nst - 2), n1 = n0 + 1;
    // the scheduling barriers keep each half of the pair in the order
    // written (left alone, the scheduler sinks the prefetches to the end)
    const word4 bh0 = bload(st, 0), bl0 = bload(st, 1), bh1 = bload(st + 1, 0), bl1 = bload(st + 1, 1);
    kstep(h0, l0, bh0, bl0);
    h0 = gload(n0, 0);
    l0 = gload(n0, 1);
    __builtin_amdgcn_sched_barrier(0);
    kstep(h1, l1, bh1, bl1);
    h1 = gload(n1, 0);
    l1 = gload(n1, 1);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// p of rows 32 w + 8 g + 4 kk + t (t = 0..3), probe li, from the split tile,
// unscaled by the probe exponent sp
__device__ __forceinline__ void tile_p4(const uint32_t* bt, int ny, int w, int g, int lane, int sw, int sp,
                                        float2 (&p)[4]) {
  const int li = lane % 32, kk = lane / 32;
  const uint32_t* brow = bt + li * ny;
  const int off = ((8 * w + 2 * g + kk) ^ (li & sw)) << 2;
  const word4 ph = *reinterpret_cast<const word4*>(brow + off);
  const word4 pl = *reinterpret_cast<const word4*>(brow + kTile * ny + off);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float2 h = unpack_h2(ph[t]), l = unpack_h2(pl[t]);
    p[t] = make_float2(ldexpf(h.x + l.x, -sp), ldexpf(h.y + l.y, -sp));
  }
}

template <int MODE, bool SMALL>
__global__ __launch_bounds__(SMALL ? 640 : 1024, SMALL ? 5 : 1) void k_cart1d_gram16(Cart1dArgs a,
                                                                                    const word4* __restrict__ G16,
                                                                                    const int* __restrict__ gexp,
                                                                                    int* __restrict__ pexp) {
  extern __shared__ float2 pt[];                   // split p tile, then the FP32 q tile, then reduction
  uint32_t* bt = reinterpret_cast<uint32_t*>(pt);  // [32][ny] hi words, then [32][ny] lo words
  const int ny = a.ny, nw = ny / 32;
  const int sw = (ny / 4) % 16 == 0 ? 15 : 7;      // chunk swizzle within the row's 16-chunk groups
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int ntiles = (a.K + kTile - 1) / kTile;
  const int b = blockIdx.x, xcd = b % 8, rest = b / 8;
  const int tile = rest % ntiles, col = xcd + 8 * (rest / ntiles);
  if (col >= a.nx) return;
  const int k0 = tile * kTile;
  constexpr int kRowsPerLane = SMALL ? 5 : 8;      // rows y = lane + 64 m of a column (ny <= 320 / 512)
  int* __restrict__ pe = pexp + ((size_t)col * ntiles + tile) * kTile;   // probe scale exponents

  // ---- prologue: wave w prepares probes j = w, w + nw, ...
  for (int j = w; j < kTile; j += nw) split_column<MODE, kRowsPerLane>(a, bt, pe, j, k0, col, lane, sw);
  __syncthreads();   // the tile and the probe exponents (global, this workgroup's) are complete

  const int li = lane % 32, kk = lane / 32;
  floatx16 accR, accI;
  tile_product(bt, G16, col, w, nw, ny, lane, sw, accR, accI);

  // ---- q = 2^-(gexp + pexp) acc + lam p on the wave's own rows, with the
  // (Re p^H q, |q|^2) partials
  const int sp = pe[li];
  const int sq = -(gexp[col] + sp);
  double d1 = 0.0, d2 = 0.0;   // q replaces acc in place
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    float2 p[4];
    tile_p4(bt, ny, w, g, lane, sw, sp, p);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int v = 4 * g + t;
      const float2 q = make_float2(fmaf(a.lam, p[t].x, ldexpf(accR[v], sq)), fmaf(a.lam, p[t].y, ldexpf(accI[v], sq)));
      d1 += (double)p[t].x * q.x + (double)p[t].y * q.y;
      d2 += (double)q.x * q.x + (double)q.y * q.y;
      accR[v] = q.x;
      accI[v] = q.y;
    }
  }
  d1 += __shfl_xor(d1, 32, 64);   // both halves of the wave hold probe li
  d2 += __shfl_xor(d2, 32, 64);
  __syncthreads();   // every wave is done with the split tile: the FP32 q tile replaces it
#pragma unroll
  for (int v = 0; v < 16; ++v) pt[tile_at(32 * w + 8 * (v / 4) + 4 * kk + (v % 4), li)] = make_float2(accR[v], accI[v]);
  __syncthreads();

  gram_finish<MODE, kRowsPerLane>(a, pt, k0, col, w, nw, lane, d1, d2);
}

size_t gram_bytes(int ny, int nx) { return (size_t)nx * ny * ny * sizeof(float2); }

bool gram_supported(int ny) { return ny % 32 == 0 && ny >= 64 && ny <= 512; }

// c(d) = sum_k w_k exp(2 pi i k d / ny) in FP64 on the host, uploaded on s
// (the caller synchronizes s before the host vector would go out of scope:
// the copy is waited for here)
static hipError_t upload_circulant(const float* maskw_h, int ny, double2* cvec_d, hipStream_t s) {
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
  const hipError_t e = hipMemcpyAsync(cvec_d, cv.data(), ny * sizeof(double2), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);   // cv leaves scope
}

// the blocks from the circulant and the maps
hipError_t build_gram(const float2* maps, const float* maskw_h, int nc, int ny, int nx, float2* G,
                      double2* cvec_d, hipStream_t s) {
  hipError_t e = upload_circulant(maskw_h, ny, cvec_d, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)(((long)ny * ny + 255) / 256), nx), block(256);
  hipLaunchKernelGGL(k_build_gram, grid, block, 0, s, maps, cvec_d, G, nc, ny);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);
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

size_t gram16_pexp_count(int nx, int K) { return (size_t)nx * ((K + kTile - 1) / kTile) * kTile; }

hipError_t build_gram16(const float2* maps, const float* maskw_h, int nc, int ny, int nx, uint32_t* G16, int* gexp,
                        double2* cvec_d, hipStream_t s) {
  hipError_t e = upload_circulant(maskw_h, ny, cvec_d, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram16_scale, dim3(nx), dim3(256), 0, s, maps, cvec_d, gexp, nc, ny);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nthr = (ny / 32) * (ny / 8) * 64;
  dim3 grid((unsigned)((nthr + 255) / 256), nx), block(256);
  hipLaunchKernelGGL(k_gram16_build, grid, block, 0, s, maps, cvec_d, gexp, reinterpret_cast<word4*>(G16), nc, ny);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

template <bool SMALL>
static hipError_t launch_gram16(int mode, const Cart1dArgs& a, const word4* G16, const int* gexp, int* pexp,
                                hipStream_t s) {
  const int nw = a.ny / 32;
  const size_t lds = (size_t)a.ny * kTile * sizeof(float2);
  if (mode < 0 || mode > 3) return hipErrorInvalidValue;
  static const hipError_t attr = [] {
    const void* fn[4] = {(const void*)k_cart1d_gram16<C1_FIRST_PROBE, SMALL>,
                         (const void*)k_cart1d_gram16<C1_FIRST_BUF, SMALL>,
                         (const void*)k_cart1d_gram16<C1_ITER, SMALL>, (const void*)k_cart1d_gram16<C1_APPLY, SMALL>};
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
    case C1_FIRST_PROBE:
      hipLaunchKernelGGL((k_cart1d_gram16<C1_FIRST_PROBE, SMALL>), grid, block, lds, s, a, G16, gexp, pexp);
      break;
    case C1_FIRST_BUF:
      hipLaunchKernelGGL((k_cart1d_gram16<C1_FIRST_BUF, SMALL>), grid, block, lds, s, a, G16, gexp, pexp);
      break;
    case C1_ITER: hipLaunchKernelGGL((k_cart1d_gram16<C1_ITER, SMALL>), grid, block, lds, s, a, G16, gexp, pexp); break;
    default: hipLaunchKernelGGL((k_cart1d_gram16<C1_APPLY, SMALL>), grid, block, lds, s, a, G16, gexp, pexp); break;
  }
  return hipGetLastError();
}

hipError_t launch_cart1d_gram16(int mode, const Cart1dArgs& a, const uint32_t* G16, const int* gexp, int* pexp,
                                hipStream_t s) {
  if (!gram_supported(a.ny)) return hipErrorInvalidValue;
  const word4* g = reinterpret_cast<const word4*>(G16);
  if (a.ny <= 320) return launch_gram16<true>(mode, a, g, gexp, pexp, s);
  return launch_gram16<false>(mode, a, g, gexp, pexp, s);
}

}  // namespace pico
