// Kaiser-Bessel gridding NUFFT for non-Cartesian operators (Sec. 3.2.2, 3.3):
// the data path (A x and A^H y per coil; PMR replicas) and, on request, the
// gridding normal operator A^H A of the CG solves.
//
// Grid G = sigma N per axis, image placed at grid index r mod G (r centred),
// plain 2-D FFT on the grid, W x W separable Kaiser-Bessel taps per sample at
// k = floor(kappa) - W/2 + 1 + t (kappa = w G / 2 pi), de-apodisation by the
// kernel's Fourier transform at r / G, scale N^-1/2.  The adjoint is the
// exact adjoint: spread with the same weights, inverse FFT, crop.
//
// Spread (A^H): samples are sorted once per operator into bins of 8 x 8 grid
// cells by the cell of their first tap.  A one-wave workgroup owns one 8 x 8
// tile of the output grid and gathers the contributions of the samples of
// its bin and of the three bins below and left of it (the only ones whose
// W-wide footprints reach the tile, W <= 8): their values (read or drawn) are
// compacted into LDS in bin order, and every lane sums, for its own grid
// point, the samples that cover it in that order.  Each grid point is written
// once, by its own tile, so the spread is deterministic and needs no atomics
// and no halo pass.
//
// Normal operator (A^H A): interpolation followed by the spread is P^H P on
// the grid, a real symmetric operator whose row for grid point g has
// nonzeros only at offsets d in [-(W-1), W-1]^2: S[g][d] = sum_m w_m(g)
// w_m(g + d).  It is built once per operator in FP64 (from the same tap
// tables) and applied per 16 x 16 grid tile with the input window (tile plus
// a W - 1 halo) in LDS and the tile's stencil in registers, for a run of
// probes; tiles that no sample's footprint reaches are written as zeros.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "arena.h"
#include "device_common.h"
#include "runtime.h"

namespace pico {

// ------------------------------------------------------------------ host tables
namespace {

double bessel_i0(double x) {   // power series sum ((x/2)^2)^k / (k!)^2
  const double q = 0.25 * x * x;
  double term = 1.0, s = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * k);
    s += term;
    if (term <= 1e-17 * s) break;
  }
  return s;
}

double kb_phi(double u, int W, double beta) {
  const double a = 1.0 - (2.0 * u / W) * (2.0 * u / W);
  return a >= 0.0 ? bessel_i0(beta * std::sqrt(a)) : 0.0;
}

double kb_phi_hat(double nu, int W, double beta) {   // continuous transform of kb_phi
  const double z2 = beta * beta - (M_PI * W * nu) * (M_PI * W * nu);
  if (z2 > 1e-12) {
    const double z = std::sqrt(z2);
    return W * std::sinh(z) / z;
  }
  if (z2 < -1e-12) {
    const double z = std::sqrt(-z2);
    return W * std::sin(z) / z;
  }
  return W;
}

}  // namespace

double kb_beta(double sigma, int W) {
  return M_PI * std::sqrt((W / sigma) * (W / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
}

size_t KbLayout::bytes_of(size_t i) const { return sizes[i]; }

KbLayout kb_layout(long M, int W, int ny, int nx, int Gy, int Gx, int K, bool normal) {
  KbLayout L;
  const size_t nb = (size_t)(Gy / kKbTile) * (Gx / kKbTile);
  const size_t s[KbLayout::kParts] = {
      (size_t)M * 4,                       // sky0
      (size_t)M * 4,                       // skx0
      (size_t)M * W * 4,                   // swy
      (size_t)M * W * 4,                   // swx
      (size_t)M * 4,                       // perm
      (nb + 1) * 4,                        // bin_ptr
      (size_t)ny * 4,                      // dy
      (size_t)nx * 4,                      // dx
      (size_t)Gx * 8,                      // twiddles x
      (size_t)Gy * 8,                      // twiddles y
      (size_t)K * Gy * Gx * 8,             // grid [K][Gy][Gx]
      normal ? (size_t)K * Gy * Gx * 8 : 0,   // grid2 [K][Gy][Gx]
      normal ? OffsetArena::round_up((size_t)(Gy / kKbStencilTile) * (Gx / kKbStencilTile) * 4) +  // tile list
                   (size_t)Gy * Gx * (2 * W - 1) * (2 * W - 1) * 4                               // stencil
             : 0,
  };
  for (int i = 0; i < KbLayout::kParts; ++i) L.sizes[i] = s[i];
  return L;
}

void kb_build_host(const float* traj_h, long M, int W, double sigma, int ny, int nx, int Gy, int Gx,
                   std::vector<int>& sky0, std::vector<int>& skx0, std::vector<float>& swy,
                   std::vector<float>& swx, std::vector<int>& perm, std::vector<int>& bin_ptr,
                   std::vector<float>& dy, std::vector<float>& dx) {
  const double beta = kb_beta(sigma, W);
  std::vector<int> ky0(M), kx0(M);
  std::vector<float> wy((size_t)M * W), wx((size_t)M * W);
  auto taps = [&](double w, int G, int& k0m, float* wt) {
    const double kappa = w * G / (2.0 * M_PI);
    const long k0 = (long)std::floor(kappa) - W / 2 + 1;
    for (int t = 0; t < W; ++t) wt[t] = (float)kb_phi(kappa - (double)(k0 + t), W, beta);
    k0m = (int)(((k0 % G) + G) % G);
  };
  for (long m = 0; m < M; ++m) {
    taps((double)traj_h[2 * m], Gy, ky0[m], &wy[(size_t)m * W]);
    taps((double)traj_h[2 * m + 1], Gx, kx0[m], &wx[(size_t)m * W]);
  }
  // counting sort by bin of the first tap (stable: sample order within a bin)
  const int nbx = Gx / kKbTile, nby = Gy / kKbTile;
  auto bin_of = [&](long m) { return (ky0[m] / kKbTile) * nbx + kx0[m] / kKbTile; };
  bin_ptr.assign((size_t)nby * nbx + 1, 0);
  for (long m = 0; m < M; ++m) ++bin_ptr[bin_of(m) + 1];
  for (size_t b = 0; b + 1 < bin_ptr.size(); ++b) bin_ptr[b + 1] += bin_ptr[b];
  std::vector<int> fill(bin_ptr.begin(), bin_ptr.end() - 1);
  perm.resize(M);
  sky0.resize(M);
  skx0.resize(M);
  swy.resize((size_t)M * W);
  swx.resize((size_t)M * W);
  for (long m = 0; m < M; ++m) {
    const int j = fill[bin_of(m)]++;
    perm[j] = (int)m;
    sky0[j] = ky0[m];
    skx0[j] = kx0[m];
    for (int t = 0; t < W; ++t) {
      swy[(size_t)j * W + t] = wy[(size_t)m * W + t];
      swx[(size_t)j * W + t] = wx[(size_t)m * W + t];
    }
  }
  dy.resize(ny);
  dx.resize(nx);
  for (int y = 0; y < ny; ++y) dy[y] = (float)(1.0 / kb_phi_hat((double)(y - ny / 2) / Gy, W, beta));
  for (int x = 0; x < nx; ++x) dx[x] = (float)(1.0 / kb_phi_hat((double)(x - nx / 2) / Gx, W, beta));
}

void kb_build_stencil(const std::vector<int>& sky0, const std::vector<int>& skx0, const std::vector<float>& swy,
                      const std::vector<float>& swx, long M, int W, int Gy, int Gx, std::vector<int>& tile_list,
                      int& n_active, std::vector<float>& stencil) {
  // S[g][d] = sum_m w_m(g) w_m(g + d): the weight of input grid point g + d
  // in output point g of P^H P, d in [-(W-1), W-1]^2, w_m the sample's taps
  constexpr int T = kKbStencilTile;
  const int D = 2 * W - 1, nty = Gy / T, ntx = Gx / T, ntiles = nty * ntx;
  std::vector<int> slot(ntiles, -1);
  for (long m = 0; m < M; ++m)   // tiles any footprint reaches are active
    for (int a = 0; a < W; ++a)
      for (int b = 0; b < W; ++b) {
        const int gy = (sky0[m] + a) % Gy, gx = (skx0[m] + b) % Gx;
        slot[(gy / T) * ntx + gx / T] = 0;
      }
  tile_list.clear();
  for (int t = 0; t < ntiles; ++t)
    if (slot[t] == 0) {
      slot[t] = (int)tile_list.size();
      tile_list.push_back(t);
    }
  n_active = (int)tile_list.size();
  for (int t = 0; t < ntiles; ++t)
    if (slot[t] < 0) tile_list.push_back(t);
  std::vector<double> acc((size_t)n_active * D * D * T * T, 0.0);
  for (long m = 0; m < M; ++m) {
    const float* wy = &swy[(size_t)m * W];
    const float* wx = &swx[(size_t)m * W];
    for (int a1 = 0; a1 < W; ++a1) {
      const int gy = (sky0[m] + a1) % Gy;
      for (int b1 = 0; b1 < W; ++b1) {
        const int gx = (skx0[m] + b1) % Gx;
        const int t = slot[(gy / T) * ntx + gx / T];
        const size_t pt = (size_t)(gy % T) * T + gx % T;
        const double w1 = (double)wy[a1] * wx[b1];
        double* base = &acc[(size_t)t * D * D * T * T + pt];
        for (int a2 = 0; a2 < W; ++a2) {
          const double w12 = w1 * wy[a2];
          const int dy = a2 - a1 + W - 1;
          for (int b2 = 0; b2 < W; ++b2) base[((size_t)dy * D + (b2 - b1 + W - 1)) * T * T] += w12 * wx[b2];
        }
      }
    }
  }
  stencil.resize(acc.size());
  for (size_t i = 0; i < acc.size(); ++i) stencil[i] = (float)acc[i];
}

// ------------------------------------------------------------------ kernels

enum KbSrc : int { KB_READ = 0, KB_NOISE = 1 };

// One 8 x 8 tile of the output grid per one-wave workgroup (blockIdx.x),
// probe blockIdx.y: gout[k][tile] = sum over the samples whose footprint
// covers each point of weight x value, the samples taken from the tile's bin
// and the three bins below / left of it, in bin order.  Sample values:
//   KB_READ    src[k * bstride + m] (m the sample's index),
//   KB_NOISE   CN(0, 1) Philox draw (stream 1, element c M + m, draw first + k).
template <int W, int SRC>
__global__ __launch_bounds__(64) void k_kb_tile_spread(KbOp o, const float2* __restrict__ src, long bstride, int c,
                                                       uint64_t seed, uint64_t first, float2* __restrict__ gout) {
  constexpr int T = kKbTile, CH = T * T, REACH = T + W - 1;
  static_assert(CH == 64, "one output point per lane of one wave");
  __shared__ float2 sv[CH];
  __shared__ int soff[CH];        // oy | ox << 16: first tap relative to the tile origin - (W - 1)
  __shared__ float sw[CH][2 * W];
  const int ty = blockIdx.x / o.nbx, tx = blockIdx.x % o.nbx, k = blockIdx.y;
  const int y0 = ty * T, x0 = tx * T, wy0 = y0 - (W - 1), wx0 = x0 - (W - 1);
  const long G2 = (long)o.Gy * o.Gx;
  const int lane = threadIdx.x, py = lane / T, px = lane % T;
  float2 acc = make_float2(0.f, 0.f);
  for (int nb = 0; nb < 4; ++nb) {
    int by = ty - 1 + (nb >> 1), bx = tx - 1 + (nb & 1);
    by += by < 0 ? o.nby : 0;
    bx += bx < 0 ? o.nbx : 0;
    const int bin = by * o.nbx + bx;
    const int p0 = o.bin_ptr[bin], p1 = o.bin_ptr[bin + 1];
    for (int c0 = p0; c0 < p1; c0 += CH) {
      const int j = c0 + lane;
      bool take = false;
      int oy = 0, ox = 0;
      if (j < p1) {
        oy = o.sky0[j] - wy0;
        ox = o.skx0[j] - wx0;
        oy += oy < 0 ? o.Gy : 0;
        oy -= oy >= o.Gy ? o.Gy : 0;
        ox += ox < 0 ? o.Gx : 0;
        ox -= ox >= o.Gx ? o.Gx : 0;
        take = oy < REACH && ox < REACH;   // the footprint meets the tile
      }
      // compaction that keeps bin order
      const uint64_t mask = __ballot(take);
      const int total = __popcll(mask);
      if (take) {
        const int pos = __popcll(mask & ((1ull << lane) - 1ull));
        float2 v;
        if constexpr (SRC == KB_READ) v = src[(size_t)k * bstride + o.perm[j]];
        else v = draw_probe(seed, first + k, (uint32_t)((size_t)c * o.M + o.perm[j]), 1u, 3);
        sv[pos] = v;
        soff[pos] = oy | (ox << 16);
#pragma unroll
        for (int t = 0; t < W; ++t) {
          sw[pos][t] = o.swy[(size_t)j * W + t];
          sw[pos][W + t] = o.swx[(size_t)j * W + t];
        }
      }
      __syncthreads();
      for (int q = 0; q < total; ++q) {
        const int off = soff[q];
        const int dyy = py + W - 1 - (off & 0xffff), dxx = px + W - 1 - (off >> 16);
        if ((unsigned)dyy < (unsigned)W && (unsigned)dxx < (unsigned)W)
          acc = cfma(acc, sw[q][dyy] * sw[q][W + dxx], sv[q]);
      }
      __syncthreads();   // the lists are rewritten by the next chunk
    }
  }
  gout[(size_t)k * G2 + (size_t)(y0 + py) * o.Gx + x0 + px] = acc;
}

// P^H P by its stencil, one 16 x 16 tile (a slot of the tile list) and a run
// of kc probes per workgroup.  Work items (probe run, slot), slots fastest,
// go to the eight XCDs in contiguous runs (workgroup b on XCD b mod 8 takes
// item (b mod 8) * ceil(total / 8) + b / 8), so tiles that share window
// halos meet in one L2; the padding workgroups return at once.
template <int W>
__global__ __launch_bounds__(256) void k_kb_stencil(KbOp o, const float2* __restrict__ gin, float2* __restrict__ gout,
                                                    int K, int kc, int slots) {
  constexpr int T = kKbStencilTile, D = 2 * W - 1, WIN = T + D - 1;
  static_assert(T * T == 256, "one output point per thread");
  __shared__ float2 win[WIN * WIN];
  const long total = (long)slots * ((K + kc - 1) / kc), per = (total + 7) / 8;
  const long item = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= total) return;
  const int slot = (int)(item % slots), tile = o.tile_list[slot], ntx = o.Gx / T;
  const int y0 = (tile / ntx) * T, x0 = (tile % ntx) * T, wy0 = y0 - (W - 1), wx0 = x0 - (W - 1);
  const int py = threadIdx.x / T, px = threadIdx.x % T;
  const int k0 = (int)(item / slots) * kc, k1 = min(K, k0 + kc);
  const long G2 = (long)o.Gy * o.Gx;
  float2* outp = gout + (size_t)(y0 + py) * o.Gx + x0 + px;
  if (slot >= o.n_active) {   // no sample reaches this tile
    for (int k = k0; k < k1; ++k) outp[(size_t)k * G2] = make_float2(0.f, 0.f);
    return;
  }
  // window points of this thread (NW per thread), and the next probe's values
  // loaded while the current probe is computed (W <= 6: at W = 8 the 225
  // stencil weights leave no registers for them)
  constexpr int NW = (WIN * WIN + 255) / 256;
  constexpr bool PF = W <= 6;
  auto goff = [&](int i) {
    int gy = wy0 + i / WIN, gx = wx0 + i % WIN;   // the window spans less than one period
    gy += gy < 0 ? o.Gy : 0;
    gy -= gy >= o.Gy ? o.Gy : 0;
    gx += gx < 0 ? o.Gx : 0;
    gx -= gx >= o.Gx ? o.Gx : 0;
    return (long)gy * o.Gx + gx;
  };
  float2 nxt[NW];
  auto load_win = [&](int k) {
    const float2* gk = gin + (size_t)k * G2;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < WIN * WIN) nxt[j] = gk[goff(i)];
    }
  };
  if (PF && k0 < k1) load_win(k0);
  float st[D * D];
  const float* sp = o.stencil + (size_t)slot * D * D * T * T + threadIdx.x;
#pragma unroll
  for (int i = 0; i < D * D; ++i) st[i] = sp[(size_t)i * T * T];
  for (int k = k0; k < k1; ++k) {
    __syncthreads();   // every thread is done with the previous window
    if constexpr (PF) {
#pragma unroll
      for (int j = 0; j < NW; ++j)
        if (threadIdx.x + 256 * j < WIN * WIN) win[threadIdx.x + 256 * j] = nxt[j];
    } else {
      const float2* gk = gin + (size_t)k * G2;
      for (int i = threadIdx.x; i < WIN * WIN; i += 256) win[i] = gk[goff(i)];
    }
    __syncthreads();
    if (PF && k + 1 < k1) load_win(k + 1);
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dy = 0; dy < D; ++dy)
#pragma unroll
      for (int dx = 0; dx < D; ++dx) acc = cfma(acc, st[dy * D + dx], win[(py + dy) * WIN + px + dx]);
    outp[(size_t)k * G2] = acc;
  }
}

// out[b * bstride + m] = sum_{a, t} wy[a] wx[t] grid[b][ky0 + a][kx0 + t], one
// thread per sample in bin order (neighbouring threads read neighbouring cells)
template <int W>
__global__ __launch_bounds__(256) void k_kb_interp(KbOp o, const float2* __restrict__ grid, float2* __restrict__ out,
                                                   long bstride) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= o.M) return;
  const float2* gb = grid + (size_t)b * o.Gy * o.Gx;
  float2 acc = make_float2(0.f, 0.f);
  int iy = o.sky0[j];
  for (int a = 0; a < W; ++a, ++iy) {
    if (iy >= o.Gy) iy -= o.Gy;
    const float wa = o.swy[(size_t)j * W + a];
    int ix = o.skx0[j];
    for (int t = 0; t < W; ++t, ++ix) {
      if (ix >= o.Gx) ix -= o.Gx;
      acc = cfma(acc, wa * o.swx[(size_t)j * W + t], gb[(size_t)iy * o.Gx + ix]);
    }
  }
  out[(size_t)b * bstride + o.perm[j]] = acc;
}

// out[b][y][x] (= or +=) conj(S_c[y][x]) grid[b][(y - ny/2) mod Gy][(x - nx/2) mod Gx] dy dx scale
__global__ void k_kb_crop_combine(const float2* __restrict__ grid, const float2* __restrict__ Sc,
                                  const float* __restrict__ dy, const float* __restrict__ dx,
                                  float2* __restrict__ out, int ny, int nx, int Gy, int Gx, float scale,
                                  int accumulate) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= (long)ny * nx) return;
  const int y = (int)(i / nx), x = (int)(i % nx);
  const int gy = (y - ny / 2 + Gy) % Gy, gx = (x - nx / 2 + Gx) % Gx;
  const float2 v = cscale(grid[(size_t)b * Gy * Gx + (size_t)gy * Gx + gx], dy[y] * dx[x] * scale);
  const float2 t = cmulc(Sc[i], v);
  float2* o = out + (size_t)b * ny * nx + i;
  *o = accumulate ? cadd(*o, t) : t;
}

// grid[b] = S_c x[b] dy dx scale placed at (r mod G), zero elsewhere
__global__ void k_kb_expand(const float2* __restrict__ xin, const float2* __restrict__ Sc,
                            const float* __restrict__ dy, const float* __restrict__ dx,
                            float2* __restrict__ grid, int ny, int nx, int Gy, int Gx, float scale) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (g >= (long)Gy * Gx) return;
  const int gy = (int)(g / Gx), gx = (int)(g % Gx);
  const int ry = gy < ny / 2 ? gy : (gy >= Gy - ny / 2 ? gy - Gy : Gy);   // Gy: outside
  const int rx = gx < nx / 2 ? gx : (gx >= Gx - nx / 2 ? gx - Gx : Gx);
  float2 v = make_float2(0.f, 0.f);
  if (ry != Gy && rx != Gx) {
    const int y = ry + ny / 2, x = rx + nx / 2;
    const size_t i = (size_t)y * nx + x;
    v = cscale(cmul(Sc[i], xin[(size_t)b * ny * nx + i]), dy[y] * dx[x] * scale);
  }
  grid[(size_t)b * Gy * Gx + g] = v;
}

static dim3 kb_grid(long n, int K) { return dim3((unsigned)((n + 255) / 256), K); }

template <int SRC>
static hipError_t tile_spread(const KbOp& o, int K, const float2* src, long bstride, int c, uint64_t seed,
                              uint64_t first, float2* gout, hipStream_t s) {
  const dim3 grid((unsigned)(o.nby * o.nbx), K), block(64);
  switch (o.W) {
    case 2: hipLaunchKernelGGL((k_kb_tile_spread<2, SRC>), grid, block, 0, s, o, src, bstride, c, seed, first, gout); break;
    case 4: hipLaunchKernelGGL((k_kb_tile_spread<4, SRC>), grid, block, 0, s, o, src, bstride, c, seed, first, gout); break;
    case 6: hipLaunchKernelGGL((k_kb_tile_spread<6, SRC>), grid, block, 0, s, o, src, bstride, c, seed, first, gout); break;
    case 8: hipLaunchKernelGGL((k_kb_tile_spread<8, SRC>), grid, block, 0, s, o, src, bstride, c, seed, first, gout); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Probes per workgroup: a workgroup loads its tile's (2W-1)^2 stencil weights
// once (124 KB at W = 6) for its run of probes, so runs grow from 16 while
// the active tiles still give at least 2048 workgroups.
static hipError_t stencil(const KbOp& o, int K, const float2* gin, float2* gout, hipStream_t s) {
  const int slots = (o.Gy / kKbStencilTile) * (o.Gx / kKbStencilTile);
  int kc = 16;
  while (kc < 128 && (long)std::max(o.n_active, 1) * ((K + 2 * kc - 1) / (2 * kc)) >= 2048) kc *= 2;
  const long total = (long)slots * ((K + kc - 1) / kc);
  const dim3 grid((unsigned)(8 * ((total + 7) / 8))), block(256);
  switch (o.W) {
    case 2: hipLaunchKernelGGL(k_kb_stencil<2>, grid, block, 0, s, o, gin, gout, K, kc, slots); break;
    case 4: hipLaunchKernelGGL(k_kb_stencil<4>, grid, block, 0, s, o, gin, gout, K, kc, slots); break;
    case 6: hipLaunchKernelGGL(k_kb_stencil<6>, grid, block, 0, s, o, gin, gout, K, kc, slots); break;
    case 8: hipLaunchKernelGGL(k_kb_stencil<8>, grid, block, 0, s, o, gin, gout, K, kc, slots); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t interp(const KbOp& o, int K, const float2* grid, float2* out, long bstride, hipStream_t s) {
  const dim3 g = kb_grid(o.M, K), block(256);
  switch (o.W) {
    case 2: hipLaunchKernelGGL(k_kb_interp<2>, g, block, 0, s, o, grid, out, bstride); break;
    case 4: hipLaunchKernelGGL(k_kb_interp<4>, g, block, 0, s, o, grid, out, bstride); break;
    case 6: hipLaunchKernelGGL(k_kb_interp<6>, g, block, 0, s, o, grid, out, bstride); break;
    case 8: hipLaunchKernelGGL(k_kb_interp<8>, g, block, 0, s, o, grid, out, bstride); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out[K][ny][nx] = A^H of K multi-coil sample arrays: src [K][nc][M] (whitened),
// or Philox CN(0, 1) noise (src == nullptr; stream 1, element c M + m)
hipError_t kb_adjoint(const KbOp& o, const float2* maps, int nc, int K, const float2* src, uint64_t seed,
                      uint64_t first, float2* out, hipStream_t s) {
  const long n = (long)o.ny * o.nx;
  const float scale = (float)(1.0 / std::sqrt((double)n));
  for (int c = 0; c < nc; ++c) {
    hipError_t e = src ? tile_spread<KB_READ>(o, K, src + (size_t)c * o.M, (long)nc * o.M, c, 0, 0, o.grid, s)
                       : tile_spread<KB_NOISE>(o, K, nullptr, 0, c, seed, first, o.grid, s);
    if (e != hipSuccess) return e;
    if ((e = launch_fft2d(o.grid, K, o.Gy, o.Gx, true, o.twx, o.twy, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_kb_crop_combine, kb_grid(n, K), dim3(256), 0, s, o.grid, maps + (size_t)c * n,
                       o.dy, o.dx, out, o.ny, o.nx, o.Gy, o.Gx, scale, c > 0 ? 1 : 0);
  }
  return hipGetLastError();
}

// out[K][nc][M] = A x for K images x [K][ny][nx]
hipError_t kb_forward(const KbOp& o, const float2* maps, int nc, int K, const float2* x, float2* out,
                      hipStream_t s) {
  const long G2 = (long)o.Gy * o.Gx, n = (long)o.ny * o.nx;
  const float scale = (float)(1.0 / std::sqrt((double)n));
  for (int c = 0; c < nc; ++c) {
    hipLaunchKernelGGL(k_kb_expand, kb_grid(G2, K), dim3(256), 0, s, x, maps + (size_t)c * n, o.dy, o.dx,
                       o.grid, o.ny, o.nx, o.Gy, o.Gx, scale);
    hipError_t e = launch_fft2d(o.grid, K, o.Gy, o.Gx, false, o.twx, o.twy, s);
    if (e != hipSuccess) return e;
    if ((e = interp(o, K, o.grid, out + (size_t)c * o.M, (long)nc * o.M, s)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ gridding normal operator

// double sum over a 256-thread block, fixed order
__device__ double block_sum256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o2 = 128; o2 > 0; o2 >>= 1) {
    if ((int)threadIdx.x < o2) red[threadIdx.x] += red[threadIdx.x + o2];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// p of the CG step per image row (blockIdx.x = y, blockIdx.y = k), as the grid
// path's first row kernel forms it, with |r|^2 of the row in part[k][y][0]
template <int MODE>
__global__ __launch_bounds__(256) void k_kbn_pro(Grid2dArgs a) {
  __shared__ double red[256];
  const int y = blockIdx.x, k = blockIdx.y;
  const size_t row = ((size_t)k * a.ny + y) * a.nx;
  float alpha = 0.f, beta = 0.f;
  if constexpr (MODE == C1_ITER) {
    alpha = (float)a.alpha[k];
    beta = (float)a.beta[k];
  }
  double d0 = 0.0;
  for (int x = threadIdx.x; x < a.nx; x += 256) {
    const size_t i = row + x;
    if constexpr (MODE == C1_FIRST_PROBE) {
      const float2 v = draw_probe(arg_seed(a), arg_first(a) + k, (uint32_t)(y * a.nx + x), 0u, a.dist);
      a.r[i] = v;
      a.p[i] = v;
      d0 += (double)v.x * v.x + (double)v.y * v.y;
    } else if constexpr (MODE == C1_FIRST_BUF) {
      const float2 v = a.r[i];
      a.p[i] = v;
      d0 += (double)v.x * v.x + (double)v.y * v.y;
    } else if constexpr (MODE == C1_ITER) {
      const float2 po = a.p[i], qo = a.q[i], ro = a.r[i];
      const float2 xo = a.x_zero ? make_float2(0.f, 0.f) : a.x[i];
      const float2 rn = cfma(ro, -alpha, qo);
      a.x[i] = cfma(xo, alpha, po);
      a.r[i] = rn;
      a.p[i] = cfma(rn, beta, po);
      d0 += (double)rn.x * rn.x + (double)rn.y * rn.y;
    }
  }
  d0 = block_sum256(d0, red);
  if (threadIdx.x == 0) a.part[((size_t)k * a.ny + y) * 4] = d0;
}

// q = (coil sum already in q) + lam p_in, and the partial dots Re p^H q, |q|^2,
// Re r^H q of the row (r = p_in outside C1_ITER)
template <int MODE>
__global__ __launch_bounds__(256) void k_kbn_epi(Grid2dArgs a) {
  __shared__ double red[256];
  const int y = blockIdx.x, k = blockIdx.y;
  const size_t row = ((size_t)k * a.ny + y) * a.nx;
  double d1 = 0.0, d2 = 0.0, d3 = 0.0;
  for (int x = threadIdx.x; x < a.nx; x += 256) {
    const size_t i = row + x;
    const float2 pin = MODE == C1_APPLY ? cscale(a.src[i], a.scale) : a.p[i];
    const float2 q = cfma(a.q[i], a.lam, pin);
    a.q[i] = q;
    const float2 rv = MODE == C1_ITER ? a.r[i] : pin;
    d1 += (double)pin.x * q.x + (double)pin.y * q.y;
    d2 += (double)q.x * q.x + (double)q.y * q.y;
    d3 += (double)rv.x * q.x + (double)rv.y * q.y;
  }
  d1 = block_sum256(d1, red);
  d2 = block_sum256(d2, red);
  d3 = block_sum256(d3, red);
  if (threadIdx.x == 0) {
    double* pp = a.part + ((size_t)k * a.ny + y) * 4;
    pp[1] = d1;
    pp[2] = d2;
    pp[3] = d3;
  }
}

hipError_t launch_kb_normal(int mode, const Grid2dArgs& a, const KbOp& o, hipStream_t s) {
  if (!o.grid2 || !o.stencil) return hipErrorInvalidValue;
  const dim3 rows((unsigned)a.ny, a.K), block(256);
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL(k_kbn_pro<C1_FIRST_PROBE>, rows, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL(k_kbn_pro<C1_FIRST_BUF>, rows, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL(k_kbn_pro<C1_ITER>, rows, block, 0, s, a); break;
    case C1_APPLY: break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long n = (long)o.ny * o.nx;
  const float scale = (float)(1.0 / std::sqrt((double)n));
  const float2* xin = mode == C1_APPLY ? a.src : a.p;
  const float in_scale = mode == C1_APPLY ? scale * a.scale : scale;
  // per coil: image rows expanded and row-transformed ([K][ny][Gx] in
  // grid2), column transforms to the full grid, stencil, inverse column
  // transforms back to the image rows (in grid), inverse row transforms
  // cropped and combined into q
  for (int c = 0; c < a.nc; ++c) {
    const float2* Sc = a.maps + (size_t)c * n;
    if ((e = launch_kbn_rows(false, xin, Sc, o.dy, o.dx, o.grid2, a.K, o.ny, o.nx, o.Gx, in_scale, 0, o.twx, s)) !=
        hipSuccess)
      return e;
    if ((e = launch_fft_cols_crop(o.grid2, o.grid, a.K, o.ny, o.Gy, o.Gx, false, o.twy, s)) != hipSuccess) return e;
    if ((e = stencil(o, a.K, o.grid, o.grid2, s)) != hipSuccess) return e;
    if ((e = launch_fft_cols_crop(o.grid2, o.grid, a.K, o.ny, o.Gy, o.Gx, true, o.twy, s)) != hipSuccess) return e;
    if ((e = launch_kbn_rows(true, o.grid, Sc, o.dy, o.dx, a.q, a.K, o.ny, o.nx, o.Gx, scale, c > 0 ? 1 : 0, o.twx,
                             s)) != hipSuccess)
      return e;
  }
  switch (mode) {
    case C1_FIRST_PROBE: hipLaunchKernelGGL(k_kbn_epi<C1_FIRST_PROBE>, rows, block, 0, s, a); break;
    case C1_FIRST_BUF: hipLaunchKernelGGL(k_kbn_epi<C1_FIRST_BUF>, rows, block, 0, s, a); break;
    case C1_ITER: hipLaunchKernelGGL(k_kbn_epi<C1_ITER>, rows, block, 0, s, a); break;
    default: hipLaunchKernelGGL(k_kbn_epi<C1_APPLY>, rows, block, 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace pico
