// Batched conjugate gradients: K independent right-hand sides, each with its
// own step scalars (Sec. 2.1, Eq. (6); App. A, Algorithm 1, covariance step).
// Vector updates run in float32; inner products are accumulated in float64
// from exact float32 products and reduced in a fixed order, and every step
// scalar (alpha, beta, |r|^2) is float64 and stays on the device.
#include "device_common.h"
#include "runtime.h"

namespace pico {

// x += alpha p, r -= alpha q; per-block partial |r|^2.
// grid (nblk, K), block 256, each thread EPT consecutive elements per round.
__global__ __launch_bounds__(256) void k_update(UpdateArgs a) {
  const int k = blockIdx.y;
  const float alpha = (float)a.alpha[k];
  const size_t off = (size_t)k * a.n;
  float2* __restrict__ x = a.x + off;
  float2* __restrict__ r = a.r + off;
  const float2* __restrict__ p = a.p + off;
  const float2* __restrict__ q = a.q + off;
  double acc = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    const float2 pv = p[i], qv = q[i];
    float2 xv = a.first_iter ? make_float2(0.f, 0.f) : x[i];
    float2 rv = r[i];
    xv = cfma(xv, alpha, pv);
    rv = cfma(rv, -alpha, qv);
    x[i] = xv;
    r[i] = rv;
    acc += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  acc = group_sum<64>(acc);
  __shared__ double red[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) a.part[(size_t)k * a.nblk + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  dim3 grid(a.nblk, a.K), block(256);
  hipLaunchKernelGGL(k_update, grid, block, 0, s, a);
  return hipGetLastError();
}

// Step scalars per right-hand side; one wavefront per probe.
//  stage 0: rr0 = rr = sum partA[.][1]; then as stage 1
//  stage 1: alpha = rr / Re(p^H q)             (freeze on breakdown)
//  stage 2: rr' = sum partB; beta = rr' / rr   (freeze at tolerance)
struct ScalarKArgs {
  ScalarArgs s;
  const double* partA;
  int nblkA;
  const double* partB;
  int nblkB;
};

__global__ __launch_bounds__(64) void k_scalars(ScalarKArgs ka) {
  const ScalarArgs& a = ka.s;
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (a.stage <= 1) {
    for (int i = lane; i < ka.nblkA; i += 64) {
      s0 += ka.partA[((size_t)k * ka.nblkA + i) * 2 + 0];
      if (a.stage == 0) s1 += ka.partA[((size_t)k * ka.nblkA + i) * 2 + 1];
    }
  } else {
    for (int i = lane; i < ka.nblkB; i += 64) s1 += ka.partB[(size_t)k * ka.nblkB + i];
  }
  s0 = group_sum<64>(s0);
  s1 = group_sum<64>(s1);
  if (lane != 0) return;
  int st = a.state[k];
  if (a.stage == 0) {
    a.rr0[k] = s1;
    a.rr[k] = s1;
    st = CG_ACTIVE;
  }
  if (a.stage <= 1) {
    const double rr = a.rr[k];
    double alpha = 0.0;
    if (st == CG_ACTIVE) {
      if (rr == 0.0) {
        st = CG_CONVERGED;
      } else if (!(s0 > 0.0) || !isfinite(s0) || !isfinite(rr)) {
        st = CG_BREAKDOWN;
      } else {
        alpha = rr / s0;
      }
    }
    a.alpha[k] = alpha;
  } else {
    double beta = 0.0;
    if (st == CG_ACTIVE) {
      const double rr = a.rr[k];
      if (!isfinite(s1)) {
        st = CG_BREAKDOWN;
      } else {
        a.rr[k] = s1;
        if (a.tol > 0.0 && sqrt(s1 / a.rr0[k]) <= a.tol) st = CG_CONVERGED;
        else beta = s1 / rr;
      }
    }
    a.beta[k] = beta;
  }
  a.state[k] = st;
}

hipError_t launch_scalars(const ScalarArgs& a, hipStream_t s) {
  // partA / partB carried through the same struct for a single launch signature
  ScalarKArgs ka{a, a.part, a.nblk, a.part, a.nblk};
  hipLaunchKernelGGL(k_scalars, dim3(a.K), dim3(64), 0, s, ka);
  return hipGetLastError();
}

// Convergence monitor: partial sums of (s - s_ref)^2 and s_ref^2 over
// standard-deviation maps s = sqrt(max(sum / N, 0)), s_ref = sqrt(max(ref, 0));
// NRMSE = sqrt(sum / sum) is finished on the host in block order.
__global__ __launch_bounds__(256) void k_nrmse_partials(const double* __restrict__ sum, double inv,
                                                        const double* __restrict__ ref, int64_t n,
                                                        double* __restrict__ part) {
  double num = 0.0, den = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double s = sqrt(fmax(sum[i] * inv, 0.0));
    const double s0 = sqrt(fmax(ref[i], 0.0));
    num += (s - s0) * (s - s0);
    den += s0 * s0;
  }
  num = group_sum<64>(num);
  den = group_sum<64>(den);
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = num;
    red[1][w] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

hipError_t launch_nrmse_partials(const double* sum, double inv_count, const double* ref, int64_t n,
                                 double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_nrmse_partials, dim3(nblk), dim3(256), 0, s, sum, inv_count, ref, n, part);
  return hipGetLastError();
}

// var = sum / N  (App. A, Algorithm 1, last step)
__global__ void k_finalize(const double* __restrict__ sum, double* __restrict__ var, int64_t n, double inv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) var[i] = sum[i] * inv;
}

hipError_t launch_finalize(const double* sum, double* var, int64_t n, double inv, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sum, var, n, inv);
  return hipGetLastError();
}

// unbiased replica variance (sum|x|^2 - |sum x|^2 / N) / (N - 1)
__global__ void k_pmr_finalize(const double* __restrict__ sum, const double* __restrict__ sum_im,
                               const double* __restrict__ sumsq, double* __restrict__ var,
                               int64_t n, double N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) var[i] = (sumsq[i] - (sum[i] * sum[i] + sum_im[i] * sum_im[i]) / N) / (N - 1.0);
}

hipError_t launch_pmr_finalize(const double* sum, const double* sum_im, const double* sumsq,
                               double* var, int64_t n, double count, hipStream_t s) {
  hipLaunchKernelGGL(k_pmr_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sum,
                     sum_im, sumsq, var, n, count);
  return hipGetLastError();
}

}  // namespace pico
