// Register-resident Stockham FFT for one line of length N spread over a
// group of T lanes of a wavefront (gfx950: 64-wide wavefronts).
//
// Lane t of the group holds v[m] = x[t + T*m], m < P = N/T, before and after
// the transform (natural order, no bit reversal).  Pass p has radix R_p; each
// lane performs B_p = P/R_p butterflies j = t + T*b.  A butterfly reads the
// elements j + r*N/R (which are exactly the lane's own registers b + B*r),
// applies the twiddles W_{NS*R}^{r*k}, k = j mod NS, computes an R-point DFT
// in registers and scatters to (j - k)*R + k + r*NS; all passes but the last
// exchange through LDS, the last one lands back in the lane's registers.
// The first pass (NS = 1) needs no twiddles.
//
// Direction: INV = false computes sum_n x[n] e^{-2 pi i n k / N},
// INV = true the unnormalised inverse (e^{+}).
#pragma once

#include "device_common.h"

namespace pico {

// ------------------------------------------------------ in-register DFTs
template <bool INV>
__device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  const float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
  constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  const float2 t1 = cadd(a1, a2);
  const float2 t2 = csub(a1, a2);
  const float2 b = make_float2(a0.x - 0.5f * t1.x, a0.y - 0.5f * t1.y);
  const float2 d = mul_mj<INV>(make_float2(h * t2.x, h * t2.y));   // -/+ j h t2
  a0 = cadd(a0, t1);
  a1 = cadd(b, d);
  a2 = csub(b, d);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
  const float2 s13 = cadd(a1, a3), d13 = mul_mj<INV>(csub(a1, a3));
  a0 = cadd(s02, s13);
  a2 = csub(s02, s13);
  a1 = cadd(d02, d13);
  a3 = csub(d02, d13);
}

template <bool INV>
__device__ __forceinline__ void dft5(float2& a0, float2& a1, float2& a2, float2& a3, float2& a4) {
  constexpr float c1 = (float)tw_cos(1, 5), c2 = (float)tw_cos(2, 5);
  constexpr float s1 = (float)tw_sin(1, 5), s2 = (float)tw_sin(2, 5);
  const float2 t1 = cadd(a1, a4), t2 = cadd(a2, a3);
  const float2 t3 = csub(a1, a4), t4 = csub(a2, a3);
  const float2 b1 = make_float2(a0.x + c1 * t1.x + c2 * t2.x, a0.y + c1 * t1.y + c2 * t2.y);
  const float2 b2 = make_float2(a0.x + c2 * t1.x + c1 * t2.x, a0.y + c2 * t1.y + c1 * t2.y);
  const float2 d1 = mul_mj<INV>(make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y));
  const float2 d2 = mul_mj<INV>(make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y));
  a0 = cadd(a0, cadd(t1, t2));
  a1 = cadd(b1, d1);
  a4 = csub(b1, d1);
  a2 = cadd(b2, d2);
  a3 = csub(b2, d2);
}

// multiply by the compile-time twiddle W_R^{m} (sign by direction)
template <int M, int R, bool INV>
__device__ __forceinline__ float2 ctwiddle(float2 a) {
  constexpr int mm = ((M % R) + R) % R;
  if constexpr (mm == 0) {
    return a;
  } else if constexpr ((4 * mm) % R == 0) {
    constexpr int q = (4 * mm) / R;                 // quarter turns, 1..3
    if constexpr (q == 2) return make_float2(-a.x, -a.y);
    else if constexpr (q == 1) return mul_mj<INV>(a);
    else return mul_mj<!INV>(a);
  } else {
    constexpr float c = (float)tw_cos(mm, R);
    constexpr float s = INV ? (float)tw_sin(mm, R) : -(float)tw_sin(mm, R);
    return cmul(a, make_float2(c, s));
  }
}

// Split of a composite R for the in-register DFT: R = F * Q with F the
// largest power of two dividing R when R is neither a power of two nor odd
// (then gcd(F, Q) = 1), else the first of 4, 2, 3, 5 that divides R.
constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }
constexpr int pow2_part(int r) { return (r & (r - 1)) == 0 ? r : ((r & 1) ? 1 : 2 * pow2_part(r / 2)); }
constexpr int dft_split(int R) {
  return (pow2_part(R) > 1 && pow2_part(R) < R) ? pow2_part(R)
         : (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 3 == 0) ? 3 : 5;
}
// k < F Q with k = k1 (mod F), k = k2 (mod Q), for coprime F and Q
constexpr int crt_index(int k1, int k2, int F, int Q) {
  int k = k2;
  while (k % F != k1) k += Q;
  return k;
}

// R-point DFT in registers.  Composite R = F * Q:
//  - coprime F, Q (Good-Thomas prime-factor split): with n = (Q n1 + F n2)
//    mod R, W_R^{n k} = W_F^{n1 k1} W_Q^{n2 k2} for k1 = k mod F, k2 = k mod Q,
//    so X[k] = DFT_F over n1 of DFT_Q over n2, with no twiddles between the two
//    stages; both index maps are compile-time register renamings;
//  - otherwise decimation in time:
//    X[k1 + Q k2] = sum_{n1<F} W_F^{n1 k2} W_R^{n1 k1} Y_{n1}[k1],
//    Y_{n1} = DFT_Q(x[n1 + F n2]).
template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&a)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<INV>(a[0], a[1]);
  } else if constexpr (R == 3) {
    dft3<INV>(a[0], a[1], a[2]);
  } else if constexpr (R == 4) {
    dft4<INV>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 5) {
    dft5<INV>(a[0], a[1], a[2], a[3], a[4]);
  } else if constexpr (gcd_i(dft_split(R), R / dft_split(R)) == 1) {
    constexpr int F = dft_split(R), Q = R / F;
    float2 y[F][Q];
    static_for<0, F>([&](auto n1) {
      static_for<0, Q>([&](auto n2) { y[n1][n2] = a[(Q * n1 + F * n2) % R]; });
      dft<Q, INV>(y[n1]);
    });
    static_for<0, Q>([&](auto k2) {
      float2 z[F];
      static_for<0, F>([&](auto n1) { z[n1] = y[n1][k2]; });
      dft<F, INV>(z);
      static_for<0, F>([&](auto k1) { a[crt_index(k1, k2, F, Q)] = z[k1]; });
    });
  } else {
    constexpr int F = dft_split(R);
    constexpr int Q = R / F;
    static_assert(F * Q == R, "radix must factor into 2, 3, 4, 5");
    float2 y[F][Q];
    static_for<0, F>([&](auto n1) {
      static_for<0, Q>([&](auto n2) { y[n1][n2] = a[n1 + F * n2]; });
      dft<Q, INV>(y[n1]);
    });
    static_for<0, Q>([&](auto k1) {
      float2 z[F];
      static_for<0, F>([&](auto n1) {
        z[n1] = ctwiddle<n1 * k1, R, INV>(y[n1][k1]);
      });
      dft<F, INV>(z);
      static_for<0, F>([&](auto k2) { a[k1 + Q * k2] = z[k2]; });
    });
  }
}

// ------------------------------------------------------------------ plans
template <int N_, int T_, int... Rs>
struct FFTPlan {
  static constexpr int N = N_;
  static constexpr int T = T_;
  static constexpr int P = N / T;
  static constexpr int NP = sizeof...(Rs);
  static constexpr int R[NP] = {Rs...};
  static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= R[i];
    return s;
  }
  // one base twiddle per butterfly of every pass after the first
  static constexpr int tw_off(int p) {
    int s = 0;
    for (int i = 1; i < p; ++i) s += P / R[i];
    return s;
  }
  static constexpr int NTW = tw_off(NP) > 0 ? tw_off(NP) : 1;
  static constexpr bool valid() {
    int prod = 1;
    for (int i = 0; i < NP; ++i) {
      if (P % R[i] != 0) return false;
      prod *= R[i];
    }
    return prod == N && N % T == 0 && 64 % T == 0;
  }
  static_assert(valid(), "invalid FFT plan");
};

// LDS index padding: one float2 of padding every 16 entries
__device__ __forceinline__ constexpr int lds_pad(int i) { return i + (i >> 4); }
template <int N>
constexpr int lds_span() { return N + N / 16 + 1; }

// Per-lane base twiddles W_{NS R}^{k} (forward sign) for every butterfly of
// every pass after the first, read once from a table W_N^m, m < N.
template <class PL>
__device__ __forceinline__ void load_twiddles(float2 (&tw)[PL::NTW],
                                              const float2* __restrict__ table, int t) {
  static_for<1, PL::NP>([&](auto pc) {
    constexpr int p = pc;
    constexpr int R = PL::R[p];
    constexpr int NS = PL::ns(p);
    constexpr int B = PL::P / R;
    constexpr int off = PL::tw_off(p);
    constexpr int stride = PL::N / (NS * R);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + PL::T * b;
      const int k = j % NS;
      tw[off + b] = table[k * stride];
    }
  });
}

template <class PL, int p, bool INV>
__device__ __forceinline__ void fft_pass(float2 (&v)[PL::P], float2* lds, int t,
                                         const float2 (&tw)[PL::NTW]) {
  constexpr int R = PL::R[p];
  constexpr int NS = PL::ns(p);
  constexpr int B = PL::P / R;
  constexpr int T = PL::T;
  constexpr bool last = (p == PL::NP - 1);
  constexpr int off = PL::tw_off(p);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[b + B * r];
    if constexpr (NS > 1) {
      const float2 w1 = INV ? make_float2(tw[off + b].x, -tw[off + b].y) : tw[off + b];
      float2 w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        a[r] = cmul(a[r], w);
        if (r + 1 < R) w = cmul(w, w1);
      }
    }
    dft<R, INV>(a);
    if constexpr (last) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + B * r] = a[r];
    } else {
      const int j = t + T * b;
      const int k = j % NS;
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_pad(base + r * NS)] = a[r];
    }
  }
  if constexpr (!last) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PL::P; ++m) v[m] = lds[lds_pad(t + T * m)];
    __syncthreads();
  }
}

template <class PL, bool INV>
__device__ __forceinline__ void fft(float2 (&v)[PL::P], float2* lds, int t,
                                    const float2 (&tw)[PL::NTW]) {
  static_for<0, PL::NP>([&](auto pc) { fft_pass<PL, pc, INV>(v, lds, t, tw); });
}

}  // namespace pico

namespace pico {

// --------------------------------------------------------------------------
// Two-step (four-step) FFT of length N = LA * VA over a group of LA lanes.
//
// Layout A: lane a < LA holds x[a + LA*m], m < VA.
// Layout B: lane b < VA holds X[b + VA*r], r < LA.
// Forward A -> B:  Y[a][k] = DFT_VA over m of x[a + LA m]   (lane a, registers)
//                  Y[a][k] *= W_N^{a k}                      (lane a)
//                  transpose through LDS                     (one exchange)
//                  X[k + VA r] = DFT_LA over a of Y[a][k]    (lane k, registers)
// Inverse B -> A is the same chain reversed with conjugate twiddles, so one
// LDS exchange per transform and both twiddle stages use lane a's own set
// {W_N^{a k} : 0 < k < VA}.  Lanes that are idle in a step still reach every
// barrier.
template <int LA_, int VA_>
struct TwoStep {
  static constexpr int LA = LA_, VA = VA_, N = LA * VA;
  static constexpr int L = (LA > VA ? LA : VA);   // lanes per group
  static constexpr int VB = LA;                    // values per lane in layout B
  static constexpr int VMAX = (VA > LA ? VA : LA);
  static constexpr int STRIDE = LA + 1;            // padded LDS row
  static constexpr int SPAN = VA * STRIDE;
  static constexpr bool kMaskInRegs = N >= 256 && LA <= 20;   // room for LA mask weights per lane
  static constexpr bool kMapsInLds = N >= 256;     // and for N / 64 staged map values
  static constexpr bool kRowsDma = N >= 256;       // few groups: direct-to-LDS row loads
  static_assert(64 % L == 0 || L <= 64, "group must fit a wavefront");
  struct Tw { float2 w[VA]; };

  __device__ static __forceinline__ int posA(int lane, int m) { return lane + LA * m; }
  __device__ static __forceinline__ int posB(int lane, int r) { return lane + VA * r; }
  __device__ static __forceinline__ bool inA(int lane) { return lane < LA; }
  __device__ static __forceinline__ bool inB(int lane) { return lane < VA; }

  __device__ static __forceinline__ void load_tw(Tw& tw, const float2* __restrict__ table, int lane) {
    const int a = lane < LA ? lane : 0;
#pragma unroll
    for (int k = 0; k < VA; ++k) tw.w[k] = table[(a * k) % N];
  }

  // v[0..VA) in layout A  ->  v[0..LA) in layout B
  template <bool INV>
  __device__ static __forceinline__ void forward(float2 (&v)[VMAX], float2* lds, int lane, const Tw& tw) {
    if (inA(lane)) {
      float2 a[VA];
#pragma unroll
      for (int m = 0; m < VA; ++m) a[m] = v[m];
      dft<VA, INV>(a);
#pragma unroll
      for (int k = 0; k < VA; ++k) {
        const float2 w = INV ? make_float2(tw.w[k].x, -tw.w[k].y) : tw.w[k];
        lds[k * STRIDE + lane] = k ? cmul(a[k], w) : a[k];
      }
    }
    __syncthreads();
    if (inB(lane)) {
      float2 b[LA];
#pragma unroll
      for (int a = 0; a < LA; ++a) b[a] = lds[lane * STRIDE + a];
      dft<LA, INV>(b);
#pragma unroll
      for (int r = 0; r < LA; ++r) v[r] = b[r];
    }
    __syncthreads();
  }

  // v[0..LA) in layout B  ->  v[0..VA) in layout A
  template <bool INV>
  __device__ static __forceinline__ void inverse(float2 (&v)[VMAX], float2* lds, int lane, const Tw& tw) {
    if (inB(lane)) {
      float2 b[LA];
#pragma unroll
      for (int r = 0; r < LA; ++r) b[r] = v[r];
      dft<LA, INV>(b);
#pragma unroll
      for (int a = 0; a < LA; ++a) lds[lane * STRIDE + a] = b[a];
    }
    __syncthreads();
    if (inA(lane)) {
      float2 a[VA];
#pragma unroll
      for (int k = 0; k < VA; ++k) {
        const float2 z = lds[k * STRIDE + lane];
        const float2 w = INV ? make_float2(tw.w[k].x, -tw.w[k].y) : tw.w[k];
        a[k] = k ? cmul(z, w) : z;
      }
      dft<VA, INV>(a);
#pragma unroll
      for (int m = 0; m < VA; ++m) v[m] = a[m];
    }
    __syncthreads();
  }
};

// Stockham plan wrapped in the same interface (layouts A and B coincide).
template <class PL>
struct StockhamCol {
  static constexpr int N = PL::N, L = PL::T, VA = PL::P, VB = PL::P, VMAX = PL::P;
  static constexpr int SPAN = lds_span<PL::N>();
  static constexpr bool kMaskInRegs = false;
  static constexpr bool kMapsInLds = false;
  static constexpr bool kRowsDma = false;
  struct Tw { float2 w[PL::NTW]; };
  __device__ static __forceinline__ int posA(int lane, int m) { return lane + L * m; }
  __device__ static __forceinline__ int posB(int lane, int r) { return lane + L * r; }
  __device__ static __forceinline__ bool inA(int) { return true; }
  __device__ static __forceinline__ bool inB(int) { return true; }
  __device__ static __forceinline__ void load_tw(Tw& tw, const float2* __restrict__ table, int lane) {
    load_twiddles<PL>(tw.w, table, lane);
  }
  template <bool INV>
  __device__ static __forceinline__ void forward(float2 (&v)[VMAX], float2* lds, int lane, const Tw& tw) {
    fft<PL, INV>(v, lds, lane, tw.w);
  }
  template <bool INV>
  __device__ static __forceinline__ void inverse(float2 (&v)[VMAX], float2* lds, int lane, const Tw& tw) {
    fft<PL, INV>(v, lds, lane, tw.w);
  }
};

}  // namespace pico
