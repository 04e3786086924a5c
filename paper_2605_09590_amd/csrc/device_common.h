// Device-side building blocks for the PICO noise-map kernels (gfx950).
//
//  * complex float2 arithmetic,
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for probes and noise,
//  * bfloat16 storage of complex values,
//  * compile-time sines/cosines for in-register DFT constants,
//  * a compile-time loop helper.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace pico {

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cfma(float2 acc, float s, float2 a) {
  return make_float2(fmaf(s, a.x, acc.x), fmaf(s, a.y, acc.y));
}
// multiply by -j (forward) or +j (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mj(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---------------------------------------------------------------- bfloat16 storage
// A complex value as two bfloat16 halves of one 32-bit word (real in the low
// half).  Packing rounds FP32 to nearest, ties to even, with gfx950's
// v_cvt_pk_bf16_f32 (both halves in one instruction); NaN stays a NaN.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float2 v) {
  const f32x2_t f = {v.x, v.y};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}
__device__ __forceinline__ float2 unpack_bf16x2(uint32_t w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

// ---------------------------------------------------------------- Philox4x32-10
struct u32x4 { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
  constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;   // round multipliers
  constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;   // Weyl key increments
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = (uint64_t)MA * c0;
    const uint64_t pb = (uint64_t)MB * c2;
    const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)pb;
    c3 = (uint32_t)pa;
    c0 = n0;
    c2 = n2;
    k0 += WA;
    k1 += WB;
  }
  return {c0, c1, c2, c3};
}

// Probe families (0 random phase, 1 QPSK, 2 real Rademacher, 3 complex Gaussian).
// Counter = (element, draw lo, draw hi, stream), key = (seed lo, seed hi).
__device__ __forceinline__ float2 draw_probe(uint64_t seed, uint64_t draw, uint32_t elem,
                                             uint32_t stream, int dist) {
  const u32x4 w = philox4x32_10(elem, (uint32_t)draw, (uint32_t)(draw >> 32), stream,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
  float s, c;
  if (dist == 0) {
    const float f2 = (float)(w.w0 >> 8) * 0x1p-23f;        // 2 f, f = (w0 >> 8) / 2^24
    sincospif(f2, &s, &c);
    return make_float2(c, s);
  } else if (dist == 1) {
    const uint32_t q = w.w0 >> 30;
    return q == 0 ? make_float2(1.f, 0.f) : q == 1 ? make_float2(0.f, 1.f)
         : q == 2 ? make_float2(-1.f, 0.f) : make_float2(0.f, -1.f);
  } else if (dist == 2) {
    return make_float2((w.w0 >> 31) ? -1.f : 1.f, 0.f);
  } else {
    const float u1 = ((float)(w.w0 >> 8) + 1.0f) * 0x1p-24f;  // (0, 1]
    const float r = sqrtf(-logf(u1));
    const float f2 = (float)(w.w1 >> 8) * 0x1p-23f;
    sincospif(f2, &s, &c);
    return make_float2(r * c, r * s);
  }
}

// Position of a launch in the probe sequence: (seed, first) from the kernel
// arguments, or from device memory at a.tp when set (a graph replayed per
// probe tile reads them there, so one captured graph serves every tile).
template <class A>
__device__ __forceinline__ uint64_t arg_seed(const A& a) {
  return a.tp ? a.tp[0] : a.seed;
}
template <class A>
__device__ __forceinline__ uint64_t arg_first(const A& a) {
  return a.tp ? a.tp[1] : a.first;
}

// ---------------------------------------------------------------- compile-time trig
// cos / sin of 2 pi m / R in double, by Taylor series after reduction to
// (-pi, pi]; used only for in-register DFT constants.
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int n = 1; n < 18; ++n) { t *= -x * x / ((2.0 * n) * (2.0 * n + 1)); s += t; }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 18; ++n) { t *= -x * x / ((2.0 * n - 1) * (2.0 * n)); s += t; }
  return s;
}
constexpr double red_angle(long m, long R) {
  long mm = m % R;
  if (mm < 0) mm += R;
  double a = 2.0 * kPi * (double)mm / (double)R;
  if (a > kPi) a -= 2.0 * kPi;
  return a;
}
constexpr double tw_cos(long m, long R) { return taylor_cos(red_angle(m, R)); }
constexpr double tw_sin(long m, long R) { return taylor_sin(red_angle(m, R)); }

// ---------------------------------------------------------------- static_for
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(std::forward<F>(f));
  }
}

// -------------------------------------------------------------- reductions
// Sum over the G lanes of an aligned lane group (G a power of two <= 64),
// fixed butterfly order, so results are bitwise reproducible.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace pico
