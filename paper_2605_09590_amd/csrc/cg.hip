// Batched conjugate gradients: K independent right-hand sides, each with its
// own step scalars (Sec. 2.1, Eq. (6); App. A, Algorithm 1, covariance step).
// Vector updates run in float32; inner products are accumulated in float64
// from exact float32 products and reduced in a fixed order, and every step
// scalar (alpha, beta, |r|^2) is float64 and stays on the device.
#include "device_common.h"
#include "runtime.h"

namespace pico {

// Last update of a solve: x += alpha p (iteration I's step; earlier steps
// are fused into the normal-operator kernel).
__global__ __launch_bounds__(256) void k_final_x(FinalArgs a) {
  const int k = blockIdx.y;
  const float alpha = (float)a.alpha[k];
  const size_t off = (size_t)k * a.n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    const float2 xo = a.x_zero ? make_float2(0.f, 0.f) : a.x[off + i];
    a.x[off + i] = cfma(xo, alpha, a.p[off + i]);
  }
}

// tp = (seed, first): the probe-sequence position a replayed tile graph reads
__global__ void k_set_tile(uint64_t* __restrict__ tp, uint64_t seed, uint64_t first) {
  if (threadIdx.x == 0) {
    tp[0] = seed;
    tp[1] = first;
  }
}

hipError_t launch_set_tile(uint64_t* tp, uint64_t seed, uint64_t first, hipStream_t s) {
  hipLaunchKernelGGL(k_set_tile, dim3(1), dim3(64), 0, s, tp, seed, first);
  return hipGetLastError();
}

hipError_t launch_final_x(const FinalArgs& a, hipStream_t s) {
  const int nblk = (a.n + 1023) / 1024;
  dim3 grid(nblk < 1024 ? nblk : 1024, a.K), block(256);
  hipLaunchKernelGGL(k_final_x, grid, block, 0, s, a);
  return hipGetLastError();
}

// Step scalars of iteration i per right-hand side (one wavefront each), from
// the partial dots of the kernel that formed p_i and q_i = (M + lam) p_i:
//   rr_i = |r_i|^2 (measured), alpha_i = rr_i / Re(p_i^H q_i),
//   rr_{i+1} = |r_i - alpha_i q_i|^2 = rr_i - 2 alpha_i Re(r_i^H q_i) + alpha_i^2 |q_i|^2,
//   beta_i = rr_{i+1} / rr_i.
// A right-hand side freezes (alpha = beta = 0 from then on) on breakdown
// (Re p^H q <= 0 or a non-finite scalar), when rr_i = 0, and, in tolerance
// mode, once sqrt(rr_{i+1} / rr_0) <= tol (after its last step is applied).
__global__ __launch_bounds__(64) void k_scalars(ScalarArgs a) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = lane; i < a.nblk; i += 64) {
    const double* pp = a.part + ((size_t)k * a.nblk + i) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] += pp[j];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) s[j] = group_sum<64>(s[j]);
  if (lane != 0) return;
  int st = a.state[k];
  const double rr = s[0];
  if (a.first) {
    a.rr0[k] = rr;
    st = CG_ACTIVE;
  }
  double alpha = 0.0, beta = 0.0;
  if (st == CG_ACTIVE) {
    if (rr == 0.0) {
      st = CG_CONVERGED;
      a.rr[k] = 0.0;
    } else if (!(s[1] > 0.0) || !isfinite(s[1]) || !isfinite(rr)) {
      st = CG_BREAKDOWN;
    } else {
      alpha = rr / s[1];
      double rn = rr - 2.0 * alpha * s[3] + alpha * alpha * s[2];
      if (!isfinite(rn)) {
        st = CG_BREAKDOWN;
        alpha = 0.0;
      } else {
        if (rn < 0.0) rn = 0.0;
        a.rr[k] = rn;
        if (rn == 0.0 || (a.tol > 0.0 && sqrt(rn / a.rr0[k]) <= a.tol)) st = CG_CONVERGED;
        else beta = rn / rr;
      }
    }
  }
  a.alpha[k] = alpha;
  a.beta[k] = beta;
  a.state[k] = st;
}

hipError_t launch_scalars(const ScalarArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars, dim3(a.K), dim3(64), 0, s, a);
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

// Reference-free error proxy of the running map (adaptive stopping): per voxel
// the sample variance of the N per-probe terms, s2 = (sumsq - N m^2) / (N - 1),
// m = sum / N, gives the variance of m as s2 / N; through sigma = sqrt(m) the
// std map's error is s2 / (4 N m).  Partials: sum of s2 / (4 N m) and of m over
// voxels with m > 0.
__global__ __launch_bounds__(256) void k_stderr_partials(const double* __restrict__ sum,
                                                         const double* __restrict__ sumsq, double N,
                                                         int64_t n, double* __restrict__ part) {
  double num = 0.0, den = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double m = sum[i] / N;
    if (m > 0.0) {
      const double s2 = fmax((sumsq[i] - N * m * m) / (N - 1.0), 0.0);
      num += s2 / (4.0 * N * m);
      den += m;
    }
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

hipError_t launch_stderr_partials(const double* sum, const double* sumsq, double count, int64_t n,
                                  double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_stderr_partials, dim3(nblk), dim3(256), 0, s, sum, sumsq, count, n, part);
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
