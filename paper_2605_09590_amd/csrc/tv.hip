// Total-variation proximal step of the compressed-sensing reconstruction
// (FISTA with lam_TV ||grad x||_1, Sec. 3.2.3 of the paper's CS experiment)
// and its forward-mode derivative for the Jacobian probes.
//
// TV(x) = sum_pixels sqrt(|(D_y x)|^2 + |(D_x x)|^2), D = periodic forward
// differences; D^H p = p_y[y-1] - p_y[y] + p_x[x-1] - p_x[x].  The prox
// prox_{lam TV}(z) = z - lam D^H p* solves the dual over pointwise unit balls
// by Beck and Teboulle's fast gradient projection (IEEE TIP 2009), a fixed
// number of inner steps from p = r = 0, step 1/(8 lam) since ||D||^2 <= 8:
//   u = z - lam D^H r,   w = r + D u / (8 lam),   p' = P(w),
//   r = p' + th_i (p' - p),   p = p',   th_i = (s_i - 1) / s_{i+1}.
// P(w) = w / max(1, |w|) per pixel, |w| = sqrt(|w_y|^2 + |w_x|^2).
//
// Primal (FP64, once per operator): every inner step stores the projection's
// derivative data, w^ = w/|w| and 1/|w| where |w| > 1, else w^ = 0 and 1, so
// the tangent map is dP(w) dw = (dw - w^ Re(w^H dw)) / |w| for all pixels,
// with the inside / outside decision taken in FP64.  Tangent (FP32, K probes
// at once): the same steps on (dz, dr, dp) with that stored dP, two or four
// inner steps per fused kernel (u and w of a tile and its halo from LDS, the halo
// recomputed), one single-step kernel first when the count is odd.
//
// Dual fields are [image][2][ny][nx] (y component, then x component).
#include "device_common.h"
#include "runtime.h"

#include <algorithm>

namespace pico {

namespace {

// v in [-n, 2n) folded into [0, n): the halo of a tile reaches one row or
// column past the image, and tiles start inside it
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Work item of workgroup b when the launch has 8 * ceil(total / 8) of them:
// workgroups go to the eight XCDs in turn, and XCD b mod 8 takes the
// contiguous run of items starting at (b mod 8) * ceil(total / 8), in the
// order (tangent block, tile) with tiles in row order, so the halo rows and
// columns that neighbouring tiles read twice are fetched into one L2.
// Returns -1 for the padding workgroups.
__device__ __forceinline__ long xcd_item(long total) {
  const long per = (total + 7) / 8;
  const long v = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  return v < total ? v : -1;
}
static dim3 xcd_grid(long total) { return dim3((unsigned)(8 * ((total + 7) / 8))); }

// out = z - lam D^H r over B images (blockIdx.y); out may alias z
__global__ void k_tv_u64(const double2* z, const double2* __restrict__ r, double2* out, int ny, int nx,
                         double lam) {
  const long n = (long)ny * nx;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = blockIdx.y;
  const int y = (int)(i / nx), x = (int)(i - (long)y * nx);
  const int ym = y ? y - 1 : ny - 1, xm = x ? x - 1 : nx - 1;
  const double2* ry = r + (size_t)b * 2 * n;
  const double2* rx = ry + n;
  const double2 a = ry[(long)ym * nx + x], c = ry[i], d = rx[(long)y * nx + xm], e = rx[i];
  const double hx = a.x - c.x + d.x - e.x, hy = a.y - c.y + d.y - e.y;
  const double2 zv = z[(size_t)b * n + i];
  out[(size_t)b * n + i] = make_double2(fma(-lam, hx, zv.x), fma(-lam, hy, zv.y));
}

// w = r + c8 D u, p' = P(w), r = p' + th (p' - p), p = p'; stores dP data
// (what, invn: [ny*nx], image 0 only) when what is given
__global__ void k_tv_w64(const double2* __restrict__ u, double2* __restrict__ r, double2* __restrict__ p,
                         int ny, int nx, double c8, double th, float4* __restrict__ what,
                         float* __restrict__ invn) {
  const long n = (long)ny * nx;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = blockIdx.y;
  const int y = (int)(i / nx), x = (int)(i - (long)y * nx);
  const int yp = y + 1 < ny ? y + 1 : 0, xp = x + 1 < nx ? x + 1 : 0;
  const double2* ub = u + (size_t)b * n;
  const double2 u0 = ub[i], uy = ub[(long)yp * nx + x], ux = ub[(long)y * nx + xp];
  double2* ry = r + (size_t)b * 2 * n;
  double2* py = p + (size_t)b * 2 * n;
  const double2 ry0 = ry[i], rx0 = ry[n + i];
  double2 wy = make_double2(fma(c8, uy.x - u0.x, ry0.x), fma(c8, uy.y - u0.y, ry0.y));
  double2 wx = make_double2(fma(c8, ux.x - u0.x, rx0.x), fma(c8, ux.y - u0.y, rx0.y));
  const double nn = sqrt(wy.x * wy.x + wy.y * wy.y + wx.x * wx.x + wx.y * wx.y);
  float4 wh = make_float4(0.f, 0.f, 0.f, 0.f);
  float iv = 1.f;
  if (nn > 1.0) {
    const double sc = 1.0 / nn;
    wy = make_double2(wy.x * sc, wy.y * sc);
    wx = make_double2(wx.x * sc, wx.y * sc);
    wh = make_float4((float)wy.x, (float)wy.y, (float)wx.x, (float)wx.y);
    iv = (float)sc;
  }
  if (what && b == 0) {
    what[i] = wh;
    invn[i] = iv;
  }
  const double2 oy = py[i], ox = py[n + i];
  ry[i] = make_double2(fma(th, wy.x - oy.x, wy.x), fma(th, wy.y - oy.y, wy.y));
  ry[n + i] = make_double2(fma(th, wx.x - ox.x, wx.x), fma(th, wx.y - ox.y, wx.y));
  py[i] = wy;
  py[n + i] = wx;
}

__global__ void k_tv_zero64(double2* __restrict__ a, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < total) a[i] = make_double2(0.0, 0.0);
}

// One tangent inner step for a TY x TX tile and tangents k0 .. k0+kper-1:
// du = dz - lam D^H dr over the tile and its +1 halo (LDS), then
// dw = dr + c8 D du, dp' = dP(w) dw, dr' = dp' + th (dp' - dp), dp = dp'.
// dr is read from drA and written to drB (neighbours are read); dp in place.
// first: dr = dp = 0 (the step from the zero start).  Every global load of
// tangent k + 1 is issued before tangent k is computed.  Needs ny >= TY + 2
// and nx >= TX + 2 (the halo wraps at most once).
constexpr int kTY = 8, kTX = 32;
constexpr int kRy = (kTY + 2) * (kTX + 1), kRx = (kTY + 1) * (kTX + 2), kRu = (kTY + 1) * (kTX + 1);
constexpr int kPer = (kRy + 255) / 256;    // region elements per thread (2 for each region)
static_assert(kRx <= kPer * 256 && kRu <= kPer * 256, "region split");

struct TangentLoads {
  float2 ry[kPer], rx[kPer], z[kPer], py, px;
};

__device__ __forceinline__ void tv_load(TangentLoads& L, const float2* __restrict__ dz, const float2* __restrict__ drA,
                                        const float2* __restrict__ dp, int k, long n, int ny, int nx, int y0, int x0,
                                        int t, bool own, long i, bool first) {
  const float2* zk = dz + (size_t)k * n;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = t + 256 * j;
    if (e < kRu) {
      const int rr = e / (kTX + 1), cc = e - rr * (kTX + 1);
      L.z[j] = zk[(long)wrap(y0 + rr, ny) * nx + wrap(x0 + cc, nx)];
    }
  }
  if (first) return;
  const float2* ry = drA + (size_t)k * 2 * n;
  const float2* rx = ry + n;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int e = t + 256 * j;
    if (e < kRy) {
      const int rr = e / (kTX + 1), cc = e - rr * (kTX + 1);
      L.ry[j] = ry[(long)wrap(y0 - 1 + rr, ny) * nx + wrap(x0 + cc, nx)];
    }
    if (e < kRx) {
      const int rr = e / (kTX + 2), cc = e - rr * (kTX + 2);
      L.rx[j] = rx[(long)wrap(y0 + rr, ny) * nx + wrap(x0 - 1 + cc, nx)];
    }
  }
  if (own) {
    const float2* pk = dp + (size_t)k * 2 * n;
    L.py = pk[i];
    L.px = pk[n + i];
  }
}

__global__ __launch_bounds__(256) void k_tv_inner(const float2* __restrict__ dz, const float2* __restrict__ drA,
                                                  float2* __restrict__ drB, float2* __restrict__ dp,
                                                  const float4* __restrict__ what, const float* __restrict__ invn,
                                                  int ny, int nx, int K, int kper, float lam, float c8, float th,
                                                  int first) {
  __shared__ float2 sRy[kTY + 2][kTX + 1];   // dr_y rows y0-1 .. y0+TY, cols x0 .. x0+TX
  __shared__ float2 sRx[kTY + 1][kTX + 2];   // dr_x rows y0 .. y0+TY, cols x0-1 .. x0+TX
  __shared__ float2 sU[kTY + 1][kTX + 1];    // du rows y0 .. y0+TY, cols x0 .. x0+TX
  const long n = (long)ny * nx;
  const int tilesx = (nx + kTX - 1) / kTX, tiles = tilesx * ((ny + kTY - 1) / kTY);
  const long item = xcd_item((long)tiles * ((K + kper - 1) / kper));
  if (item < 0) return;
  const int tile = (int)(item % tiles), kblk = (int)(item / tiles);
  const int y0 = (tile / tilesx) * kTY, x0 = (tile % tilesx) * kTX;
  const int t = threadIdx.x, ty = t / kTX, tx = t % kTX;
  const int y = y0 + ty, x = x0 + tx;
  const bool own = y < ny && x < nx;
  const long i = (long)y * nx + x;
  const bool fst = first != 0;
  float4 wh = make_float4(0.f, 0.f, 0.f, 0.f);
  float iv = 1.f;
  if (own) {
    wh = what[i];
    iv = invn[i];
  }
  const int k0 = kblk * kper, k1 = min(K, k0 + kper);
  TangentLoads cur;
  cur.py = cur.px = make_float2(0.f, 0.f);
  if (k0 < k1) tv_load(cur, dz, drA, dp, k0, n, ny, nx, y0, x0, t, own, i, fst);
  for (int k = k0; k < k1; ++k) {
    if (!fst) {
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int e = t + 256 * j;
        if (e < kRy) {
          const int rr = e / (kTX + 1), cc = e - rr * (kTX + 1);
          sRy[rr][cc] = cur.ry[j];
        }
        if (e < kRx) {
          const int rr = e / (kTX + 2), cc = e - rr * (kTX + 2);
          sRx[rr][cc] = cur.rx[j];
        }
      }
      __syncthreads();
    }
    float2 oy = cur.py, ox = cur.px;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int e = t + 256 * j;
      if (e < kRu) {
        const int rr = e / (kTX + 1), cc = e - rr * (kTX + 1);
        float2 u = cur.z[j];
        if (!fst) {
          const float hx = sRy[rr][cc].x - sRy[rr + 1][cc].x + sRx[rr][cc].x - sRx[rr][cc + 1].x;
          const float hy = sRy[rr][cc].y - sRy[rr + 1][cc].y + sRx[rr][cc].y - sRx[rr][cc + 1].y;
          u = make_float2(fmaf(-lam, hx, u.x), fmaf(-lam, hy, u.y));
        }
        sU[rr][cc] = u;
      }
    }
    float2 ryo = make_float2(0.f, 0.f), rxo = ryo;
    if (own && !fst) {
      ryo = sRy[ty + 1][tx];
      rxo = sRx[ty][tx + 1];
    }
    __syncthreads();
    if (k + 1 < k1) tv_load(cur, dz, drA, dp, k + 1, n, ny, nx, y0, x0, t, own, i, fst);
    if (own) {
      const float2 u0 = sU[ty][tx], uy = sU[ty + 1][tx], ux = sU[ty][tx + 1];
      const float2 wy = make_float2(fmaf(c8, uy.x - u0.x, ryo.x), fmaf(c8, uy.y - u0.y, ryo.y));
      const float2 wx = make_float2(fmaf(c8, ux.x - u0.x, rxo.x), fmaf(c8, ux.y - u0.y, rxo.y));
      const float re = wh.x * wy.x + wh.y * wy.y + wh.z * wx.x + wh.w * wx.y;   // Re(w^H dw)
      const float2 qy = make_float2((wy.x - wh.x * re) * iv, (wy.y - wh.y * re) * iv);
      const float2 qx = make_float2((wx.x - wh.z * re) * iv, (wx.y - wh.w * re) * iv);
      float2* rb = drB + (size_t)k * 2 * n;
      float2* pk = dp + (size_t)k * 2 * n;
      rb[i] = make_float2(fmaf(th, qy.x - oy.x, qy.x), fmaf(th, qy.y - oy.y, qy.y));
      rb[n + i] = make_float2(fmaf(th, qx.x - ox.x, qx.x), fmaf(th, qx.y - ox.y, qx.y));
      pk[i] = qy;
      pk[n + i] = qx;
    }
    __syncthreads();
  }
}

// S tangent inner steps i .. i+S-1 in one pass over a TY x TX tile T
// (S = 2 on 8 x 32 tiles; S = 4 on 16 x 32, or 16 x 16 when fused with the
// FISTA step; one thread per pixel of T).  The box B is T grown by S on
// every side (FIN: by S + 1 above and left), index [a][b] = pixel
// (y0 - S - E + a, x0 - S - E + b), periodic, E = FIN.  Step s (from 0)
// updates r and p on R_s = rows [s+1, BY-2-s] x cols [s+1, BX-2-s] from
// u_s = dz - lam D^H r_s on U_s = R_s grown by one towards +y / +x; u_s reads
// r on R_{s-1} (the whole box for s = 0), so R_{S-1} = T (FIN: T with the row
// above and the column left of it):
//   w = r_s + c8 D u_s,  p_{s+1} = dP_s(w),  r_{s+1} = p_{s+1} + th_s (p_{s+1} - p_s).
// Thread t (of TY * TX) owns the box points e = t + TY TX j (j < NPT)
// through every step: their r, p, dz and u stay in its registers, and only r
// and u go through LDS, for the neighbours' reads (a point reads r at (a-1,
// b), (a, b-1) and u at (a+1, b), (a, b+1)).  The steps' projection data sits
// in LDS region by region, loaded once per workgroup for its run of
// tangents.  Inputs: r_i on B, p_i
// on R_0, dz on U_0, read from (rA, pA); without FIN r and p of T written to
// (rB, pB) (neighbouring tiles read the halo of both; last: the prox's last
// pass, only p is read afterwards).  FIN (the prox's last pass, fused with the
// FISTA step): nothing is written to the dual fields; each pixel of T forms
// the prox output dx = dz - lam D^H p from the box, then y = dx + theta (dx -
// xo), xo = dx.  first: r_i = p_i = 0 (step 0 from the zero start).  Tangent
// k + 1's box is loaded into registers while tangent k's steps run.  Needs
// ny >= TY + 2S + E and nx >= TX + 2S + E (the halo wraps at most once).
template <int S, int TY, int TX, int E>
struct TvSteps {
  static constexpr int BY = TY + 2 * S + E, BX = TX + 2 * S + E, NB = BY * BX;
  static constexpr int NT = TY * TX;             // threads per workgroup
  static constexpr int NPT = (NB + NT - 1) / NT; // box points per thread
  __host__ __device__ static constexpr int ry(int s) { return BY - 2 - 2 * s; }   // R_s rows
  __host__ __device__ static constexpr int rx(int s) { return BX - 2 - 2 * s; }   // R_s cols
  __host__ __device__ static constexpr int proj_off(int s) {
    int o = 0;
    for (int q = 0; q < s; ++q) o += ry(q) * rx(q);
    return o;
  }
  static constexpr int NPROJ = proj_off(S);   // projection data of the S steps on their regions
};

struct TvTheta {
  float th[4];
};

template <int S, int TY, int TX, bool FIN>
__global__ __launch_bounds__(TY * TX) void k_tv_steps(const float2* __restrict__ dz, const float2* __restrict__ rA,
                                                  float2* __restrict__ rB, const float2* __restrict__ pA,
                                                  float2* __restrict__ pB, const float4* __restrict__ what,
                                                  const float* __restrict__ invn, int ny, int nx, int K, int kper,
                                                  float lam, float c8, TvTheta th, int first, int last,
                                                  float2* __restrict__ xo, float2* __restrict__ yo, float theta) {
  constexpr int E = FIN ? 1 : 0;
  using C = TvSteps<S, TY, TX, E>;
  constexpr int BY = C::BY, BX = C::BX, NB = C::NB, NT = C::NT, NPT = C::NPT;
  __shared__ float2 sRy[BY][BX], sRx[BY][BX];   // r_s at every box point
  __shared__ float2 sU[BY][BX];                 // u_s
  __shared__ float4 sW[C::NPROJ];               // projection data of the steps on R_s (w^)
  __shared__ float sV[C::NPROJ];                // and 1/|w|
  const long n = (long)ny * nx;
  const int tilesx = (nx + TX - 1) / TX, tiles = tilesx * ((ny + TY - 1) / TY);
  const long item = xcd_item((long)tiles * ((K + kper - 1) / kper));
  if (item < 0) return;
  const int tile = (int)(item % tiles), kblk = (int)(item / tiles);
  const int y0 = (tile / tilesx) * TY, x0 = (tile % tilesx) * TX;
  const int t = threadIdx.x;
  const bool fst = first != 0;
  // this thread's box points: coordinates, in-box flag, image index
  int sa[NPT], sb[NPT], gi[NPT];   // images have fewer than 2^31 pixels
  bool sv[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int e = t + NT * j;
    sv[j] = e < NB;
    const int ee = sv[j] ? e : 0;
    sa[j] = ee / BX;
    sb[j] = ee - sa[j] * BX;
    gi[j] = wrap(y0 - S - E + sa[j], ny) * nx + wrap(x0 - S - E + sb[j], nx);
  }
  auto inU = [&](int s, int j) {
    return sv[j] && sa[j] >= s + 1 && sa[j] <= BY - 1 - s && sb[j] >= s + 1 && sb[j] <= BX - 1 - s;
  };
  auto inR = [&](int s, int j) {
    return sv[j] && sa[j] >= s + 1 && sa[j] <= BY - 2 - s && sb[j] >= s + 1 && sb[j] <= BX - 2 - s;
  };
  auto inT = [&](int j) {   // own output pixels: T, inside the image
    const int a = sa[j] - S - E, b = sb[j] - S - E;
    return sv[j] && a >= 0 && a < TY && b >= 0 && b < TX && y0 + a < ny && x0 + b < nx;
  };
  // projection data of the S steps on their regions, shared by the run of
  // tangents
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int RY = C::ry(s), RX = C::rx(s), off = C::proj_off(s);
    for (int e = t; e < RY * RX; e += NT) {
      const int a = s + 1 + e / RX, b = s + 1 + e % RX;
      const int g = wrap(y0 - S - E + a, ny) * nx + wrap(x0 - S - E + b, nx);
      sW[off + e] = what[(size_t)s * n + g];
      sV[off + e] = invn[(size_t)s * n + g];
    }
  }
  const int k0 = kblk * kper, k1 = min(K, k0 + kper);
  float2 nry[NPT], nrx[NPT], npy[NPT], npx[NPT], nz[NPT];
  auto box_load = [&](int k) {
    const float2* zk = dz + (size_t)k * n;
    const float2* ryk = rA + (size_t)k * 2 * n;
    const float2* pyk = pA + (size_t)k * 2 * n;
    const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      nry[j] = nrx[j] = npy[j] = npx[j] = nz[j] = zero;
      if (!fst) {
        nry[j] = ryk[gi[j]];
        nrx[j] = ryk[n + gi[j]];
        if (inR(0, j)) {
          npy[j] = pyk[gi[j]];
          npx[j] = pyk[n + gi[j]];
        }
      }
      if (inU(0, j)) nz[j] = zk[gi[j]];
    }
  };
  if (k0 < k1) box_load(k0);
  for (int k = k0; k < k1; ++k) {
    float2 ry[NPT], rx[NPT], py[NPT], px[NPT], zz[NPT], uu[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
      ry[j] = nry[j];
      rx[j] = nrx[j];
      py[j] = npy[j];
      px[j] = npx[j];
      zz[j] = nz[j];
      uu[j] = make_float2(0.f, 0.f);
      if (sv[j]) {
        sRy[sa[j]][sb[j]] = ry[j];
        sRx[sa[j]][sb[j]] = rx[j];
      }
    }
    __syncthreads();
    if (k + 1 < k1) box_load(k + 1);   // in flight during this tangent's steps
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int j = 0; j < NPT; ++j) {   // u_s = dz - lam D^H r_s on U_s
        if (inU(s, j)) {
          const int a = sa[j], b = sb[j];
          const float2 ryn = sRy[a - 1][b], rxn = sRx[a][b - 1];
          const float hx = ryn.x - ry[j].x + rxn.x - rx[j].x;
          const float hy = ryn.y - ry[j].y + rxn.y - rx[j].y;
          uu[j] = make_float2(fmaf(-lam, hx, zz[j].x), fmaf(-lam, hy, zz[j].y));
          sU[a][b] = uu[j];
        }
      }
      __syncthreads();
      const float ths = th.th[s];
#pragma unroll
      for (int j = 0; j < NPT; ++j) {   // step s on R_s: w, dP(w) dw, r and p
        if (inR(s, j)) {
          const int a = sa[j], b = sb[j];
          const float2 uy = sU[a + 1][b], ux = sU[a][b + 1];
          const float2 wy = make_float2(fmaf(c8, uy.x - uu[j].x, ry[j].x), fmaf(c8, uy.y - uu[j].y, ry[j].y));
          const float2 wx = make_float2(fmaf(c8, ux.x - uu[j].x, rx[j].x), fmaf(c8, ux.y - uu[j].y, rx[j].y));
          const int pe = C::proj_off(s) + (a - s - 1) * C::rx(s) + (b - s - 1);
          const float4 wh = sW[pe];
          const float iv = sV[pe];
          const float re = wh.x * wy.x + wh.y * wy.y + wh.z * wx.x + wh.w * wx.y;   // Re(w^H dw)
          const float2 qy = make_float2((wy.x - wh.x * re) * iv, (wy.y - wh.y * re) * iv);
          const float2 qx = make_float2((wx.x - wh.z * re) * iv, (wx.y - wh.w * re) * iv);
          ry[j] = make_float2(fmaf(ths, qy.x - py[j].x, qy.x), fmaf(ths, qy.y - py[j].y, qy.y));
          rx[j] = make_float2(fmaf(ths, qx.x - px[j].x, qx.x), fmaf(ths, qx.y - px[j].y, qx.y));
          py[j] = qy;
          px[j] = qx;
          if (s + 1 < S) {   // r_{s+1} for the next step's neighbour reads
            sRy[a][b] = ry[j];
            sRx[a][b] = rx[j];
          } else if (FIN) {   // p_S for the prox output's neighbour reads
            sRy[a][b] = qy;
            sRx[a][b] = qx;
          }
        }
      }
      if (s + 1 < S || FIN) __syncthreads();
    }
    if constexpr (FIN) {
#pragma unroll
      for (int j = 0; j < NPT; ++j) {   // prox output and FISTA step on T
        if (inT(j)) {
          const int a = sa[j], b = sb[j];
          const float2 pyn = sRy[a - 1][b], pxn = sRx[a][b - 1];
          const float hx = pyn.x - py[j].x + pxn.x - px[j].x;
          const float hy = pyn.y - py[j].y + pxn.y - px[j].y;
          const float2 dxv = make_float2(fmaf(-lam, hx, zz[j].x), fmaf(-lam, hy, zz[j].y));
          const size_t o = (size_t)k * n + gi[j];
          const float2 xp = xo[o];
          yo[o] = make_float2(fmaf(theta, dxv.x - xp.x, dxv.x), fmaf(theta, dxv.y - xp.y, dxv.y));
          xo[o] = dxv;
        }
      }
      __syncthreads();   // the next tangent's r overwrites these p values
    } else {
      float2* rb = rB + (size_t)k * 2 * n;
      float2* pb = pB + (size_t)k * 2 * n;
#pragma unroll
      for (int j = 0; j < NPT; ++j) {
        if (inT(j)) {
          if (!last) {   // the prox's last pass: only p is read afterwards
            rb[gi[j]] = ry[j];
            rb[n + gi[j]] = rx[j];
          }
          pb[gi[j]] = py[j];
          pb[n + gi[j]] = px[j];
        }
      }
    }
  }
}

// dx = dz - lam D^H dp; y = dx + theta (dx - xo); xo = dx   (K images)
__global__ void k_tv_final(const float2* __restrict__ dz, const float2* __restrict__ dp, float2* __restrict__ xo,
                           float2* __restrict__ yo, int ny, int nx, float lam, float theta) {
  const long n = (long)ny * nx;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = blockIdx.y;
  const int y = (int)(i / nx), x = (int)(i - (long)y * nx);
  const int ym = y ? y - 1 : ny - 1, xm = x ? x - 1 : nx - 1;
  const float2* py = dp + (size_t)k * 2 * n;
  const float2* px = py + n;
  const float2 a = py[(long)ym * nx + x], c = py[i], d = px[(long)y * nx + xm], e = px[i];
  const size_t o = (size_t)k * n + i;
  const float2 zv = dz[o];
  const float2 dx = make_float2(fmaf(-lam, a.x - c.x + d.x - e.x, zv.x), fmaf(-lam, a.y - c.y + d.y - e.y, zv.y));
  const float2 b = xo[o];
  yo[o] = make_float2(fmaf(theta, dx.x - b.x, dx.x), fmaf(theta, dx.y - b.y, dx.y));
  xo[o] = dx;
}

dim3 grid_img(long n, int B) { return dim3((unsigned)((n + 255) / 256), (unsigned)B); }

}  // namespace

hipError_t tv64_prox(const Cs64& o, int B, double2* z, double lam, float4* what, float* invn, hipStream_t s) {
  if (lam == 0.0) return hipSuccess;
  const long n = (long)o.ny * o.nx;
  const long dual = 2 * n * B;
  hipLaunchKernelGGL(k_tv_zero64, grid_img(dual, 1), dim3(256), 0, s, o.tv_r, dual);
  hipLaunchKernelGGL(k_tv_zero64, grid_img(dual, 1), dim3(256), 0, s, o.tv_p, dual);
  const double c8 = 1.0 / (8.0 * lam);
  for (int it = 0; it < o.tv_inner; ++it) {
    hipLaunchKernelGGL(k_tv_u64, grid_img(n, B), dim3(256), 0, s, z, o.tv_r, o.tv_u, o.ny, o.nx, lam);
    hipLaunchKernelGGL(k_tv_w64, grid_img(n, B), dim3(256), 0, s, o.tv_u, o.tv_r, o.tv_p, o.ny, o.nx, c8,
                       o.tv_th[it], what ? what + (size_t)it * n : nullptr, what ? invn + (size_t)it * n : nullptr);
  }
  hipLaunchKernelGGL(k_tv_u64, grid_img(n, B), dim3(256), 0, s, z, o.tv_p, z, o.ny, o.nx, lam);
  return hipGetLastError();
}

template <int S, int TY, int TX, bool FIN>
static void launch_tv_steps(const float2* dz, float2* drA, float2* drB, float2* dpA, float2* dpB, const float4* what,
                            const float* invn, const float* th, int ny, int nx, int K, float lam, float c8, int first,
                            int last, float2* xo, float2* yo, float theta, hipStream_t s) {
  const int tiles = ((ny + TY - 1) / TY) * ((nx + TX - 1) / TX);
  int kper = 8;
  while (kper > 1 && (long)tiles * ((K + kper - 1) / kper) < 2048) kper >>= 1;
  const dim3 grid = xcd_grid((long)tiles * ((K + kper - 1) / kper));
  TvTheta tt{};
  for (int q = 0; q < S; ++q) tt.th[q] = th[q];
  hipLaunchKernelGGL((k_tv_steps<S, TY, TX, FIN>), grid, dim3(TY * TX), 0, s, dz, drA, drB, dpA, dpB, what, invn, ny, nx,
                     K, kper, lam, c8, tt, first, last, xo, yo, theta);
}

constexpr int kFY = 16, kFX = 32;   // four-step tiles (512 threads)

hipError_t tv_tangent_step(const float2* dz, float2* drA, float2* drB, float2* dpA, float2* dpB,
                           const float4* what, const float* invn, int ny, int nx, int K, int inner,
                           const float* th, float lam, float2* xo, float2* yo, float theta, hipStream_t s) {
  if (ny < kTY + 5 || nx < kTX + 5) return hipErrorInvalidValue;
  const long n = (long)ny * nx;
  const int tiles = ((ny + kTY - 1) / kTY) * ((nx + kTX - 1) / kTX);
  int kper = 8;
  while (kper > 1 && (long)tiles * ((K + kper - 1) / kper) < 2048) kper >>= 1;
  const dim3 grid = xcd_grid((long)tiles * ((K + kper - 1) / kper));
  const float c8 = 1.0f / (8.0f * lam);
  int it = 0;
  if (inner & 1) {   // an odd count starts with one single step (dp updated in place)
    hipLaunchKernelGGL(k_tv_inner, grid, dim3(256), 0, s, dz, drA, drB, dpA, what, invn, ny, nx, K, kper, lam, c8,
                       th[0], 1);
    std::swap(drA, drB);
    it = 1;
  }
  // four steps per pass while four remain (kFY x kFX tiles, halo 4; a last
  // pass of four, fused with the FISTA step, on 16 x 16 tiles, halo 5 above
  // and left: its larger box would leave one workgroup per CU), then pairs;
  // the last pass ends with the FISTA step
  const bool four = ny >= kFY + 9 && nx >= kFX + 9;
  for (; four && inner - it >= 4; it += 4) {
    const int fst = it == 0 ? 1 : 0;
    if (it + 4 == inner)
      launch_tv_steps<4, 16, 16, true>(dz, drA, drB, dpA, dpB, what + (size_t)it * n, invn + (size_t)it * n, th + it,
                                       ny, nx, K, lam, c8, fst, 1, xo, yo, theta, s);
    else
      launch_tv_steps<4, kFY, kFX, false>(dz, drA, drB, dpA, dpB, what + (size_t)it * n, invn + (size_t)it * n,
                                        th + it, ny, nx, K, lam, c8, fst, 0, nullptr, nullptr, 0.f, s);
    std::swap(drA, drB);
    std::swap(dpA, dpB);
  }
  for (; it < inner; it += 2) {
    const int fst = it == 0 ? 1 : 0;
    if (it + 2 >= inner)
      launch_tv_steps<2, kTY, kTX, true>(dz, drA, drB, dpA, dpB, what + (size_t)it * n, invn + (size_t)it * n,
                                         th + it, ny, nx, K, lam, c8, fst, 1, xo, yo, theta, s);
    else
      launch_tv_steps<2, kTY, kTX, false>(dz, drA, drB, dpA, dpB, what + (size_t)it * n, invn + (size_t)it * n,
                                          th + it, ny, nx, K, lam, c8, fst, 0, nullptr, nullptr, 0.f, s);
    std::swap(drA, drB);
    std::swap(dpA, dpB);
  }
  if (inner == 1)   // the single step alone: the FISTA step as its own pass
    hipLaunchKernelGGL(k_tv_final, grid_img(n, K), dim3(256), 0, s, dz, dpA, xo, yo, ny, nx, lam, theta);
  return hipGetLastError();
}

}  // namespace pico
