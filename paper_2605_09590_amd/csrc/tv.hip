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
// at once): the same steps on (dz, dr, dp) with that stored dP, two inner
// steps per fused kernel (u and w of a tile and its halo from LDS, the halo
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
  const int tilesx = (nx + kTX - 1) / kTX;
  const int y0 = (int)(blockIdx.x / tilesx) * kTY, x0 = (int)(blockIdx.x % tilesx) * kTX;
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
  const int k0 = blockIdx.y * kper, k1 = min(K, k0 + kper);
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

// Two tangent inner steps i and i+1 in one pass over a TY x TX tile T:
// step i on T grown by one pixel on every side (B1), then step i+1 on T.
// Inputs on the grown boxes (LDS, coordinates of the box B2 = T grown by 2,
// index [a][b] = pixel (y0 - 2 + a, x0 - 2 + b), periodic):
//   r_i on B2, p_i on B1, dz on B1 grown by one towards +y / +x.
// Step i:   u_i = dz - lam D^H r_i (B1 and its +y / +x neighbours),
//           p_{i+1} = dP_i(r_i + c8 D u_i), r_{i+1} = p_{i+1} + th_i (p_{i+1} - p_i)   on B1;
// step i+1: u_{i+1} on T and its +y / +x neighbours, then p_{i+2}, r_{i+2} on T.
// r and p are read from (rA, pA) and written to (rB, pB): neighbouring tiles
// read the halo of both.  first: r_i = p_i = 0 (step 0 from the zero start).
// Needs ny >= TY + 4 and nx >= TX + 4 (the halo wraps at most once).
constexpr int kBY = kTY + 4, kBX = kTX + 4;         // box B2
constexpr int kB2 = kBY * kBX;

__global__ __launch_bounds__(256) void k_tv_inner2(const float2* __restrict__ dz, const float2* __restrict__ rA,
                                                   float2* __restrict__ rB, const float2* __restrict__ pA,
                                                   float2* __restrict__ pB, const float4* __restrict__ what0,
                                                   const float* __restrict__ invn0, const float4* __restrict__ what1,
                                                   const float* __restrict__ invn1, int ny, int nx, int K, int kper,
                                                   float lam, float c8, float th0, float th1, int first) {
  __shared__ float2 sRy[kBY][kBX], sRx[kBY][kBX];   // r_i, then r_{i+1} (in place)
  __shared__ float2 sPy[kBY][kBX], sPx[kBY][kBX];   // p_i, then p_{i+1} (in place)
  __shared__ float2 sZ[kBY][kBX];                   // dz
  __shared__ float2 sU[kBY][kBX];                   // u_i, then u_{i+1}
  __shared__ float4 sW[kBY][kBX];                   // projection data of step i (w^)
  __shared__ float sV[kBY][kBX];                    // and 1/|w|
  const long n = (long)ny * nx;
  const int tilesx = (nx + kTX - 1) / kTX;
  const int y0 = (int)(blockIdx.x / tilesx) * kTY, x0 = (int)(blockIdx.x % tilesx) * kTX;
  const int t = threadIdx.x;
  const bool fst = first != 0;
  auto gidx = [&](int a, int b) { return (long)wrap(y0 - 2 + a, ny) * nx + wrap(x0 - 2 + b, nx); };
  // projection data of step i on B1 (box rows / cols 1 .. TY+2 / TX+2), shared by all tangents
  for (int e = t; e < kB2; e += 256) {
    const int a = e / kBX, b = e - a * kBX;
    if (a >= 1 && a <= kTY + 2 && b >= 1 && b <= kTX + 2) {
      const long g = gidx(a, b);
      sW[a][b] = what0[g];
      sV[a][b] = invn0[g];
    }
  }
  // own pixel: step i+1's projection data
  const int ty = t / kTX, tx = t % kTX;
  const int y = y0 + ty, x = x0 + tx;
  const bool own = y < ny && x < nx;
  const long i = (long)y * nx + x;
  float4 wh1 = make_float4(0.f, 0.f, 0.f, 0.f);
  float iv1 = 1.f;
  if (own) {
    wh1 = what1[i];
    iv1 = invn1[i];
  }
  const int k0 = blockIdx.y * kper, k1 = min(K, k0 + kper);
  // phase A: a tangent's box values (r on B2, p on B1, dz on rows / cols >= 1)
  // for this thread's points e = t, t + 256; tangent k + 1's are loaded into
  // registers while tangent k's phases run, and stored to LDS at the top of
  // the next pass
  static_assert(kB2 <= 512, "two box points per thread");
  struct BoxPt {
    float2 vy, vx, qy, qx, z;
  };
  BoxPt nb[2];
  auto box_load = [&](int k) {
    const float2* zk = dz + (size_t)k * n;
    const float2* ry = rA + (size_t)k * 2 * n;
    const float2* py = pA + (size_t)k * 2 * n;
    const float2 zero = make_float2(0.f, 0.f);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int e = t + 256 * it;
      nb[it].vy = nb[it].vx = nb[it].qy = nb[it].qx = nb[it].z = zero;
      if (e < kB2) {
        const int a = e / kBX, b = e - a * kBX;
        const long g = gidx(a, b);
        if (!fst) {
          nb[it].vy = ry[g];
          nb[it].vx = ry[n + g];
          if (a >= 1 && a <= kTY + 2 && b >= 1 && b <= kTX + 2) {
            nb[it].qy = py[g];
            nb[it].qx = py[n + g];
          }
        }
        if (a >= 1 && b >= 1) nb[it].z = zk[g];
      }
    }
  };
  if (k0 < k1) box_load(k0);
  for (int k = k0; k < k1; ++k) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int e = t + 256 * it;
      if (e < kB2) {
        const int a = e / kBX, b = e - a * kBX;
        sRy[a][b] = nb[it].vy;
        sRx[a][b] = nb[it].vx;
        sPy[a][b] = nb[it].qy;
        sPx[a][b] = nb[it].qx;
        sZ[a][b] = nb[it].z;
      }
    }
    __syncthreads();
    if (k + 1 < k1) box_load(k + 1);   // in flight during this tangent's phases
    // phase B: u_i on rows / cols 1 .. TY+3 / TX+3
    for (int e = t; e < kB2; e += 256) {
      const int a = e / kBX, b = e - a * kBX;
      if (a >= 1 && b >= 1) {
        const float hx = sRy[a - 1][b].x - sRy[a][b].x + sRx[a][b - 1].x - sRx[a][b].x;
        const float hy = sRy[a - 1][b].y - sRy[a][b].y + sRx[a][b - 1].y - sRx[a][b].y;
        sU[a][b] = make_float2(fmaf(-lam, hx, sZ[a][b].x), fmaf(-lam, hy, sZ[a][b].y));
      }
    }
    __syncthreads();
    // phase C: step i on B1; r and p replaced in place (each point reads only itself)
    for (int e = t; e < kB2; e += 256) {
      const int a = e / kBX, b = e - a * kBX;
      if (a >= 1 && a <= kTY + 2 && b >= 1 && b <= kTX + 2) {
        const float2 u0 = sU[a][b], uy = sU[a + 1][b], ux = sU[a][b + 1];
        const float2 wy = make_float2(fmaf(c8, uy.x - u0.x, sRy[a][b].x), fmaf(c8, uy.y - u0.y, sRy[a][b].y));
        const float2 wx = make_float2(fmaf(c8, ux.x - u0.x, sRx[a][b].x), fmaf(c8, ux.y - u0.y, sRx[a][b].y));
        const float4 wh = sW[a][b];
        const float iv = sV[a][b];
        const float re = wh.x * wy.x + wh.y * wy.y + wh.z * wx.x + wh.w * wx.y;
        const float2 qy = make_float2((wy.x - wh.x * re) * iv, (wy.y - wh.y * re) * iv);
        const float2 qx = make_float2((wx.x - wh.z * re) * iv, (wx.y - wh.w * re) * iv);
        const float2 oy = sPy[a][b], ox = sPx[a][b];
        sRy[a][b] = make_float2(fmaf(th0, qy.x - oy.x, qy.x), fmaf(th0, qy.y - oy.y, qy.y));
        sRx[a][b] = make_float2(fmaf(th0, qx.x - ox.x, qx.x), fmaf(th0, qx.y - ox.y, qx.y));
        sPy[a][b] = qy;
        sPx[a][b] = qx;
      }
    }
    __syncthreads();
    // phase D: u_{i+1} on rows / cols 2 .. TY+2 / TX+2 (T and its +y / +x neighbours)
    for (int e = t; e < kB2; e += 256) {
      const int a = e / kBX, b = e - a * kBX;
      if (a >= 2 && a <= kTY + 2 && b >= 2 && b <= kTX + 2) {
        const float hx = sRy[a - 1][b].x - sRy[a][b].x + sRx[a][b - 1].x - sRx[a][b].x;
        const float hy = sRy[a - 1][b].y - sRy[a][b].y + sRx[a][b - 1].y - sRx[a][b].y;
        sU[a][b] = make_float2(fmaf(-lam, hx, sZ[a][b].x), fmaf(-lam, hy, sZ[a][b].y));
      }
    }
    __syncthreads();
    // phase E: step i+1 on T, written out
    if (own) {
      const int a = ty + 2, b = tx + 2;
      const float2 u0 = sU[a][b], uy = sU[a + 1][b], ux = sU[a][b + 1];
      const float2 wy = make_float2(fmaf(c8, uy.x - u0.x, sRy[a][b].x), fmaf(c8, uy.y - u0.y, sRy[a][b].y));
      const float2 wx = make_float2(fmaf(c8, ux.x - u0.x, sRx[a][b].x), fmaf(c8, ux.y - u0.y, sRx[a][b].y));
      const float re = wh1.x * wy.x + wh1.y * wy.y + wh1.z * wx.x + wh1.w * wx.y;
      const float2 qy = make_float2((wy.x - wh1.x * re) * iv1, (wy.y - wh1.y * re) * iv1);
      const float2 qx = make_float2((wx.x - wh1.z * re) * iv1, (wx.y - wh1.w * re) * iv1);
      const float2 oy = sPy[a][b], ox = sPx[a][b];
      float2* rb = rB + (size_t)k * 2 * n;
      float2* pb = pB + (size_t)k * 2 * n;
      rb[i] = make_float2(fmaf(th1, qy.x - oy.x, qy.x), fmaf(th1, qy.y - oy.y, qy.y));
      rb[n + i] = make_float2(fmaf(th1, qx.x - ox.x, qx.x), fmaf(th1, qx.y - ox.y, qx.y));
      pb[i] = qy;
      pb[n + i] = qx;
    }
    __syncthreads();
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

hipError_t tv_tangent_prox(const float2* dz, float2* drA, float2* drB, float2* dpA, float2* dpB,
                           const float4* what, const float* invn, int ny, int nx, int K, int inner,
                           const float* th, float lam, float2** dp_out, hipStream_t s) {
  if (ny < kTY + 4 || nx < kTX + 4) return hipErrorInvalidValue;
  const long n = (long)ny * nx;
  const int tiles = ((ny + kTY - 1) / kTY) * ((nx + kTX - 1) / kTX);
  int kper = 8;
  while (kper > 1 && (long)tiles * ((K + kper - 1) / kper) < 2048) kper >>= 1;
  const dim3 grid((unsigned)tiles, (unsigned)((K + kper - 1) / kper));
  const float c8 = 1.0f / (8.0f * lam);
  int it = 0;
  if (inner & 1) {   // an odd count starts with one single step (dp updated in place)
    hipLaunchKernelGGL(k_tv_inner, grid, dim3(256), 0, s, dz, drA, drB, dpA, what, invn, ny, nx, K, kper, lam, c8,
                       th[0], 1);
    std::swap(drA, drB);
    it = 1;
  }
  for (; it < inner; it += 2) {
    hipLaunchKernelGGL(k_tv_inner2, grid, dim3(256), 0, s, dz, drA, drB, dpA, dpB, what + (size_t)it * n,
                       invn + (size_t)it * n, what + (size_t)(it + 1) * n, invn + (size_t)(it + 1) * n, ny, nx, K,
                       kper, lam, c8, th[it], th[it + 1], it == 0 ? 1 : 0);
    std::swap(drA, drB);
    std::swap(dpA, dpB);
  }
  *dp_out = dpA;
  return hipGetLastError();
}

hipError_t tv_tangent_final(const float2* dz, const float2* dp, float2* xo, float2* yo, int ny, int nx, int K,
                            float lam, float theta, hipStream_t s) {
  hipLaunchKernelGGL(k_tv_final, grid_img((long)ny * nx, K), dim3(256), 0, s, dz, dp, xo, yo, ny, nx, lam, theta);
  return hipGetLastError();
}

}  // namespace pico
