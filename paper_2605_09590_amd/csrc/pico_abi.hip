// Host runtime behind the C ABI in include/pico.h.
//
// Owns the operator (whitened maps, sampling weights, twiddle tables, the
// batched-CG workspace) and sequences the kernels of one probe tile:
//   probe tile -> K independent CG solves (App. A, Algorithm 1, covariance
//   step) -> FP64 accumulation of conj(v) . u.
// Two operator layouts share the driver:
//   separable Cartesian (phase-encode mask): one fused column kernel per
//     normal-operator application, per-probe fields column-major [K][nx][ny];
//   2-D grid (Cartesian 2-D mask, non-Cartesian Toeplitz): three kernels per
//     application, per-probe fields row-major [K][ny][nx].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "arena.h"
#include "pico.h"
#include "runtime.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

pico_status_t fail(pico_status_t st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_OR_RETURN(expr)                                                          \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(PICO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace pico {

namespace {
std::mutex g_alloc_mu;
DevAllocator g_alloc;   // guarded by g_alloc_mu; both NULL: hipMalloc / hipFree
}  // namespace

hipError_t dev_alloc(void** ptr, size_t bytes, DevAllocator* by) {
  DevAllocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
  }
  *by = a;
  *ptr = nullptr;
  if (!a.alloc) return hipMalloc(ptr, bytes);
  void* p = a.alloc(bytes, a.ctx);
  if (!p) return hipErrorOutOfMemory;
  if (reinterpret_cast<uintptr_t>(p) % OffsetArena::kAlign) {
    a.free(p, a.ctx);
    return hipErrorInvalidValue;
  }
  *ptr = p;
  return hipSuccess;
}

void dev_free(void* ptr, const DevAllocator& by) {
  if (!ptr) return;
  if (by.free) by.free(ptr, by.ctx);
  else (void)hipFree(ptr);
}

}  // namespace pico

struct pico_op_s {
  int ny = 0, nx = 0, nc = 0, sampling = 0, recon = 0;
  int reduce_f = 0;           // reduced-grid operator: coarsening factor (0 = native)
  int cg_iters = 0, K = 0;
  double cg_tol = 0.0, lam_rel = 0.0, lam_abs = 0.0;
  bool colmajor = true;       // separable Cartesian layout
  int Gy = 0, Gx = 0;         // 2-D grid size
  int nblk = 0;               // partial-dot blocks per probe (nx or ny)
  hipStream_t last_stream = nullptr;
  // resident operator
  float2* maps = nullptr;     // whitened maps (layout per path)
  uint32_t* maps_bf = nullptr;  // bfloat16 storage: the same maps packed (maps then hold the rounded values)
  bool stream_bf = false;     // grid path: row-transformed planes T kept as bfloat16
  float* maskw = nullptr;     // separable path: [ny] mask[k] / ny
  bool use_gram = false;      // separable path: dense per-column blocks on the matrix cores
  float2* gram = nullptr;     // [nx][ny][ny] conj(M_x[i][j]) at [x][j][i]
  double2* gram_c = nullptr;  // [ny] circulant c(d) (build input)
  bool use_gram16 = false;    // the same blocks split into FP16 pairs (FP16 matrix cores)
  uint32_t* gram16 = nullptr; // [nx][ny/32][ny/8][hi, lo][64 lanes][4] packed FP16 pairs
  int* gram16_exp = nullptr;  // [nx] block scale exponents
  int* gram16_pexp = nullptr; // [nx][tiles][32] probe scale exponents (kernel scratch)
  float2* twt = nullptr;      // separable path: [ny] twiddles
  float* w = nullptr;         // grid path: [Gx][Gy] real weights
  float2* twx = nullptr;      // grid path: [Gx] twiddles
  float2* twy = nullptr;      // grid path: [Gy] twiddles
  float2* T = nullptr;        // grid path: [K][nc][ny][Gx]
  // batched CG workspace, K images each
  float2 *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double* part = nullptr;     // [K][nblk][4] partial dots
  double* mon = nullptr;      // [512] convergence-monitor partials
  double *alpha = nullptr, *beta = nullptr, *rr = nullptr, *rr0 = nullptr;
  int* state = nullptr;
  // compressed sensing (FISTA + L1 wavelet or TV)
  bool cs = false;
  int fista_T = 0, levels = 0;
  int tv_inner = 0;                 // TV prox steps (0: wavelet prox)
  std::vector<double> tv_th64;      // dual momentum weights of the TV prox
  std::vector<float> tv_th;
  float4* tv_what = nullptr;        // [T][inner][ny][nx] projection data of the primal
  float* tv_invn = nullptr;         // [T][inner][ny][nx]
  float2 *tv_dp = nullptr, *tv_dpB = nullptr, *tv_drA = nullptr, *tv_drB = nullptr;  // [K][2][ny][nx] dual tangents
  double cs_lam = 0.0;
  double s2 = 0.0;              // 1.01 lambda_max(M)
  std::vector<float> theta;     // FISTA momentum weights (tangents)
  float2 *wA = nullptr, *wB = nullptr;  // wavelet buffers, K images
  double2* ctraj = nullptr;     // [T][ny][nx] stored Psi z_k of the FP64 primal
  float2* xrec = nullptr;       // reconstruction
  std::vector<double> theta64;  // FISTA momentum weights (FP64 primal)
  pico::Cs64 c64;               // FP64 operator of the primal (maps, DFT matrices)
  double2 *atb64 = nullptr, *x64 = nullptr;   // A^H b and x_T in FP64
  // replica workspace of pico_pmr_cs, allocated on its first call
  int pmr_B = 0;
  double2 *pmr_atb = nullptr, *pmr_y = nullptr, *pmr_x = nullptr, *pmr_z = nullptr, *pmr_tmp = nullptr,
          *pmr_q = nullptr, *pmr_tv_r = nullptr, *pmr_tv_p = nullptr, *pmr_tv_u = nullptr;
  uint8_t* mask_d = nullptr;    // [ny][nx] (Cartesian 2-D)
  // Kaiser-Bessel gridding data path (non-Cartesian, kb_width > 0)
  bool has_kb = false;
  bool kb_normal = false;       // CG normal operator by gridding (A_grid^H A_grid) instead of Toeplitz
  pico::KbOp kb;
  // device memory: from the allocator in effect (pico_set_allocator, else
  // hipMalloc), or from a serving arena when one is set; bytes are counted in
  // 256-byte pieces (current and peak)
  struct Alloc {
    void* ptr;
    size_t bytes;
    pico::DevAllocator by;
  };
  pico::DeviceArena* arena = nullptr;
  std::vector<Alloc> allocs;
  size_t bytes = 0, peak = 0;
  // probe tiles replayed from HIP graphs (desc.graph): one captured kernel
  // sequence per (tile size, probe family, accumulator buffers); (seed, first)
  // of the replayed tile in tile_par
  struct TileGraph {
    int K, dist;
    const double *sum, *sum_im, *sumsq;
    hipGraphExec_t exec;
    uint64_t used;
  };
  bool use_graph = false;
  uint64_t* tile_par = nullptr;   // device [2]
  hipStream_t cap_stream = nullptr;
  std::vector<TileGraph> graphs;
  uint64_t graph_clock = 0;
  // optional per-kernel-class timing with HIP events on the caller's stream
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_recs;

  ~pico_op_s() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& a : allocs) free_raw(a);
  }
  void free_raw(const Alloc& a) {
    if (arena) arena->release(a.ptr);
    else pico::dev_free(a.ptr, a.by);
  }
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }
  template <class T>
  hipError_t alloc(T** ptr, size_t count) {
    const size_t nb = pico::OffsetArena::round_up(count * sizeof(T));
    void* raw = nullptr;
    pico::DevAllocator by;
    if (arena) {
      raw = arena->alloc(nb);
      if (!raw) return hipErrorOutOfMemory;
    } else {
      hipError_t e = pico::dev_alloc(&raw, nb, &by);
      if (e != hipSuccess) return e;
    }
    allocs.push_back({raw, nb, by});
    bytes += nb;
    peak = std::max(peak, bytes);
    *ptr = static_cast<T*>(raw);
    return hipSuccess;
  }
  void release(void* ptr) {
    auto it = std::find_if(allocs.begin(), allocs.end(), [&](const Alloc& a) { return a.ptr == ptr; });
    if (it != allocs.end()) {
      free_raw(*it);
      bytes -= it->bytes;
      allocs.erase(it);
    }
  }
  size_t image() const { return (size_t)ny * nx; }
};

namespace {

// Cholesky L L^H = psi (lower), then L^-1; float64 on the host.
bool cholesky_inverse(const double* psi, int n, std::vector<double>& linv_out, std::string& why) {
  std::vector<cd> A(n * n), L(n * n, cd(0, 0)), Li(n * n, cd(0, 0));
  for (int i = 0; i < n * n; ++i) A[i] = cd(psi[2 * i], psi[2 * i + 1]);
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(A[i * n + i]));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (std::abs(A[i * n + j] - std::conj(A[j * n + i])) > 1e-10 * scale) {
        why = "psi is not Hermitian";
        return false;
      }
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[j * n + k]);
    if (!(d > 0.0)) {
      why = "psi is not positive definite";
      return false;
    }
    const double ljj = std::sqrt(d);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cd s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * std::conj(L[j * n + k]);
      L[i * n + j] = s / ljj;
    }
  }
  for (int j = 0; j < n; ++j) {  // forward substitution for each unit vector
    Li[j * n + j] = 1.0 / L[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      cd s = 0.0;
      for (int k = j; k < i; ++k) s -= L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = s / L[i * n + i];
    }
  }
  linv_out.resize(2 * n * n);
  for (int i = 0; i < n * n; ++i) {
    linv_out[2 * i] = Li[i].real();
    linv_out[2 * i + 1] = Li[i].imag();
  }
  return true;
}

std::vector<float2> twiddle_table(int n) {
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double ang = -2.0 * 3.14159265358979323846 * (double)m / (double)n;
    tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  return tw;
}

pico_status_t check_op(pico_op_t op) {
  if (!op) return fail(PICO_EINVAL, "NULL operator handle");
  return PICO_OK;
}

// Run one launch, bracketed by HIP events when profiling is on.
template <class F>
hipError_t timed(pico_op_t op, int kind, hipStream_t s, F&& launch) {
  if (!op->prof_on) return launch();
  hipEvent_t a = op->next_event(), b = op->next_event();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if ((e = hipEventRecord(b, s)) != hipSuccess) return e;
  op->prof_recs.push_back({kind, {a, b}});
  return hipSuccess;
}

// One application of the normal operator to K probes.
struct NormalCall {
  uint64_t seed = 0, first = 0;
  const uint64_t* tp = nullptr;   // graph replay: (seed, first) in device memory
  int dist = 0;
  const float2* src = nullptr;  // C1_APPLY input
  float2* dst = nullptr;        // C1_APPLY output (default q)
  float lam = 0.0f;
  float scale = 1.0f;
  int x_zero = 0;
};

hipError_t launch_normal(pico_op_t op, int K, int mode, const NormalCall& c, hipStream_t s) {
  if (op->colmajor) {
    pico::Cart1dArgs a{};
    a.ny = op->ny;
    a.nx = op->nx;
    a.nc = op->nc;
    a.K = K;
    a.maps = op->maps;
    a.maps_bf = op->maps_bf;
    a.maskw = op->maskw;
    a.twt = op->twt;
    a.src = c.src;
    a.x = op->x;
    a.r = op->r;
    a.p = op->p;
    a.q = c.dst ? c.dst : op->q;
    a.alpha = op->alpha;
    a.beta = op->beta;
    a.x_zero = c.x_zero;
    a.part = op->part;
    a.lam = c.lam;
    a.scale = c.scale;
    a.seed = c.seed;
    a.first = c.first;
    a.tp = c.tp;
    a.dist = c.dist;
    if (op->use_gram && mode != pico::C1_PMR_RHS) return pico::launch_cart1d_gram(mode, a, op->gram, s);
    if (op->use_gram16 && mode != pico::C1_PMR_RHS)
      return pico::launch_cart1d_gram16(mode, a, op->gram16, op->gram16_exp, op->gram16_pexp, s);
    return pico::launch_cart1d(mode, a, s);
  }
  pico::Grid2dArgs g{};
  g.ny = op->ny;
  g.nx = op->nx;
  g.nc = op->nc;
  g.K = K;
  g.Gy = op->Gy;
  g.Gx = op->Gx;
  g.maps = op->maps;
  g.maps_bf = op->maps_bf;
  g.w = op->w;
  g.twx = op->twx;
  g.twy = op->twy;
  g.T = op->T;
  g.Tb = op->stream_bf ? reinterpret_cast<uint32_t*>(op->T) : nullptr;
  g.src = c.src;
  g.x = op->x;
  g.r = op->r;
  g.p = op->p;
  g.q = c.dst ? c.dst : op->q;
  g.alpha = op->alpha;
  g.beta = op->beta;
  g.x_zero = c.x_zero;
  g.part = op->part;
  g.lam = c.lam;
  g.scale = c.scale;
  g.seed = c.seed;
  g.first = c.first;
  g.tp = c.tp;
  g.dist = c.dist;
  if (op->kb_normal) return pico::launch_kb_normal(mode, g, op->kb, s);
  return pico::launch_grid_normal(mode, g, s);
}

hipError_t scalars(pico_op_t op, int K, bool first, hipStream_t s) {
  pico::ScalarArgs sa{};
  sa.K = K;
  sa.part = op->part;
  sa.nblk = op->nblk;
  sa.alpha = op->alpha;
  sa.beta = op->beta;
  sa.rr = op->rr;
  sa.rr0 = op->rr0;
  sa.state = op->state;
  sa.tol = op->cg_tol;
  sa.first = first ? 1 : 0;
  return timed(op, PICO_PROF_CG_SCALARS, s, [&] { return pico::launch_scalars(sa, s); });
}

// One batched CG solve of (M + lam) x = b for K right-hand sides, x0 = 0.
// Iteration i's vector update is fused into the kernels that apply the
// normal operator for iteration i + 1; the last one runs on its own.  The
// first normal-operator application uses ``first_mode`` (probe draw or the
// right-hand side already in r); the solution ends in op->x.
hipError_t cg_solve(pico_op_t op, int K, int first_mode, uint64_t seed, uint64_t first, int dist,
                    hipStream_t s, const uint64_t* tp = nullptr) {
  NormalCall c;
  c.seed = seed;
  c.first = first;
  c.tp = tp;
  c.dist = dist;
  c.lam = (float)op->lam_abs;
  hipError_t e = timed(op, PICO_PROF_NORMAL_FIRST, s, [&] { return launch_normal(op, K, first_mode, c, s); });
  if (e != hipSuccess) return e;
  if ((e = scalars(op, K, true, s)) != hipSuccess) return e;
  for (int it = 1; it < op->cg_iters; ++it) {
    c.x_zero = (it == 1);
    if ((e = timed(op, PICO_PROF_NORMAL_ITER, s, [&] { return launch_normal(op, K, pico::C1_ITER, c, s); })) != hipSuccess) return e;
    if ((e = scalars(op, K, false, s)) != hipSuccess) return e;
  }
  pico::FinalArgs f{};
  f.n = (int)op->image();
  f.K = K;
  f.x = op->x;
  f.p = op->p;
  f.alpha = op->alpha;
  f.x_zero = (op->cg_iters == 1);   // a single step: x enters as 0
  return timed(op, PICO_PROF_CG_UPDATE, s, [&] { return pico::launch_final_x(f, s); });
}

// u = Sigma v for the K right-hand sides (probes drawn in-kernel or already
// in r): one solve for lam = 0, else solve, M, solve (Sec. 2.1, Eq. (8)).
hipError_t apply_sigma(pico_op_t op, int K, int first_mode, uint64_t seed, uint64_t first, int dist,
                       hipStream_t s, const uint64_t* tp = nullptr) {
  hipError_t e = cg_solve(op, K, first_mode, seed, first, dist, s, tp);
  if (e != hipSuccess || op->lam_abs == 0.0) return e;
  NormalCall c;
  c.src = op->x;
  c.dst = op->r;   // t = M w lands in r, the next right-hand side
  c.lam = 0.0f;
  if ((e = timed(op, PICO_PROF_OTHER, s, [&] { return launch_normal(op, K, pico::C1_APPLY, c, s); })) != hipSuccess) return e;
  return cg_solve(op, K, pico::C1_FIRST_BUF, 0, 0, 0, s);
}

hipError_t accumulate(pico_op_t op, int K, const pico_accum_t* acc, uint64_t seed, uint64_t first,
                      int dist, int pmr, hipStream_t s, const uint64_t* tp = nullptr) {
  pico::AccumArgs aa{};
  aa.ny = op->ny;
  aa.nx = op->nx;
  aa.K = K;
  aa.x = op->x;
  aa.sum = acc->sum;
  aa.sum_im = acc->sum_im;
  aa.sumsq = acc->sumsq;
  aa.seed = seed;
  aa.first = first;
  aa.tp = tp;
  aa.dist = dist;
  aa.pmr = pmr;
  return timed(op, PICO_PROF_ACCUM, s, [&] {
    return op->colmajor ? pico::launch_accum_colmajor(aa, s) : pico::launch_accum_rowmajor(aa, s);
  });
}

struct StatAcc {
  int64_t n = 0;
  double maxr = 0.0, sumr = 0.0;
  int frozen = 0;
};

hipError_t collect_stats(pico_op_t op, int K, hipStream_t s, StatAcc& sa) {
  std::vector<double> rr(K), rr0(K);
  std::vector<int> st(K);
  hipError_t e;
  if ((e = hipMemcpyAsync(rr.data(), op->rr, K * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(rr0.data(), op->rr0, K * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(st.data(), op->state, K * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  for (int k = 0; k < K; ++k) {
    const double rel = rr0[k] > 0 ? std::sqrt(std::max(rr[k], 0.0) / rr0[k]) : 0.0;
    sa.maxr = std::max(sa.maxr, rel);
    sa.sumr += rel;
    sa.frozen += (st[k] == pico::CG_BREAKDOWN);
  }
  sa.n += K;
  return hipSuccess;
}

pico_status_t write_stats(pico_op_t op, const StatAcc& sa, pico_stats_t* st) {
  st->probes = sa.n;
  st->max_relres = sa.maxr;
  st->mean_relres = sa.n ? sa.sumr / sa.n : 0.0;
  st->frozen = sa.frozen;
  st->lambda_abs = op->lam_abs;
  if (sa.frozen) return fail(PICO_ENOTCONV, "CG breakdown in " + std::to_string(sa.frozen) + " right-hand side(s)");
  return PICO_OK;
}


// lambda_max of M (Rayleigh quotient after power_iters steps from a fixed
// Philox start vector; Sec. 3.2.1, 3.3)
hipError_t power_lambda(pico_op_t op, int iters, double* out, hipStream_t s) {
  hipError_t e = op->colmajor ? pico::launch_power_start(op->p, op->ny, op->nx, s)
                              : pico::launch_power_start_rowmajor(op->p, (int)op->image(), s);
  if (e != hipSuccess) return e;
  double lam_hat = 0.0;
  float2* bufs[2] = {op->p, op->q};
  NormalCall c;
  c.lam = 0.0f;
  std::vector<double> part((size_t)op->nblk * 4);
  for (int it = 0; it < iters; ++it) {
    c.src = bufs[it & 1];
    c.dst = bufs[(it + 1) & 1];
    if ((e = launch_normal(op, 1, pico::C1_APPLY, c, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(part.data(), op->part, part.size() * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    double vq = 0.0, qq = 0.0;
    for (int b = 0; b < op->nblk; ++b) {
      vq += part[4 * b + 1];
      qq += part[4 * b + 2];
    }
    lam_hat = vq;              // Rayleigh quotient of the unit vector (scale * src)
    c.scale = (float)(1.0 / std::sqrt(qq));
  }
  *out = lam_hat;
  return hipSuccess;
}

// (-1)^((ny+nx)/2) / sqrt(ny nx): the centred orthonormal 2-D DFT's adjoint as an
// unnormalised inverse FFT between (-1)^(ky+kx) and (-1)^(y+x) sign flips
float kspace_scale(pico_op_t op) {
  const float sg = (((op->ny + op->nx) / 2) & 1) ? -1.0f : 1.0f;
  return sg / std::sqrt((float)op->image());
}

// out[K][ny][nx] = A^H of K k-space arrays (Cartesian 2-D grid operator): the
// arrays come from src (whitened with linv when given) or Philox draws
hipError_t adjoint_kspace(pico_op_t op, int K, const float2* src, const double* linv, uint64_t seed,
                          uint64_t first, uint32_t stream, int dist, float2* out, hipStream_t s,
                          const uint64_t* tp = nullptr) {
  hipError_t e = pico::launch_kspace_in(src, linv, op->mask_d, op->T, K, op->nc, op->ny, op->nx, seed,
                                        first, tp, stream, dist, kspace_scale(op), s);
  if (e != hipSuccess) return e;
  if ((e = pico::launch_fft2d(op->T, (long)K * op->nc, op->ny, op->nx, true, op->twx, op->twy, s)) != hipSuccess) return e;
  return pico::launch_coil_combine(op->T, op->maps, out, K, op->nc, (long)op->image(), s);
}

// Tangents of the T FISTA iterations for K probes at once: the gradient offset
// is A^H w (in op->r, per probe); the prox derivative is the soft threshold's
// at the stored FP64 c_k, or the TV prox's through its inner steps at the
// stored projection data.  The tangent of x_T ends in op->x.
hipError_t fista_tangent(pico_op_t op, int K, hipStream_t s) {
  const long n = (long)op->image();
  hipError_t e;
  if ((e = pico::launch_fill_zero(op->p, K * n, s)) != hipSuccess) return e;
  if ((e = pico::launch_fill_zero(op->x, K * n, s)) != hipSuccess) return e;
  NormalCall c;
  c.src = op->p;
  c.dst = op->q;
  c.lam = 0.0f;
  const float inv_s2 = (float)(1.0 / op->s2);
  for (int k = 1; k <= op->fista_T; ++k) {
    if ((e = timed(op, PICO_PROF_NORMAL_ITER, s, [&] { return launch_normal(op, K, pico::C1_APPLY, c, s); })) != hipSuccess) return e;
    e = timed(op, PICO_PROF_OTHER, s, [&] {
      hipError_t e2;
      if (op->tv_inner > 0) {
        if ((e2 = pico::launch_fista_grad(op->p, op->q, op->r, op->wA, n, K, 1, inv_s2, s)) != hipSuccess) return e2;
        // TV prox tangent at the stored projection data of iteration k
        if (op->cs_lam == 0.0) return pico::launch_momentum(op->wA, op->x, op->p, K * n, op->theta[k - 1], s);
        const size_t off = (size_t)(k - 1) * op->tv_inner * n;
        return pico::tv_tangent_step(op->wA, op->tv_drA, op->tv_drB, op->tv_dp, op->tv_dpB, op->tv_what + off,
                                     op->tv_invn + off, op->ny, op->nx, K, op->tv_inner, op->tv_th.data(),
                                     (float)op->cs_lam, op->x, op->p, (float)op->theta[k - 1], s);
      }
      // xd = Psi^H D_k(Psi zd): zd formed inside the analysis, coefficients in wB
      // (wA scratch), the synthesis applying the momentum into (x, p) directly
      const double2* ck = op->ctraj + (size_t)(k - 1) * n;
      if ((e2 = pico::launch_cs_analysis(op->p, op->q, op->r, inv_s2, op->wA, op->wB, K, op->ny, op->nx, op->levels,
                                         ck, op->cs_lam, s)) != hipSuccess)
        return e2;
      return pico::launch_cs_synthesis(op->wB, op->wA, K, op->ny, op->nx, op->levels, op->x, op->p, op->theta[k - 1], s);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// K tangents u = J w: probes drawn (src == nullptr: Philox stream 2) or given
hipError_t cs_tangents(pico_op_t op, int K, const float2* w, uint64_t seed, uint64_t first, int dist,
                       hipStream_t s, const uint64_t* tp = nullptr) {
  hipError_t e = timed(op, PICO_PROF_NORMAL_FIRST, s, [&] {
    return adjoint_kspace(op, K, w, nullptr, seed, first, 2u, dist, op->r, s, tp);
  });
  if (e != hipSuccess) return e;
  return fista_tangent(op, K, s);
}

// One probe tile of pico_noise_map: K probes from ``first`` through Sigma (or
// J for CS) and the FP64 accumulation.  tp non-NULL: the kernels read
// (seed, first) there instead (graph capture).
hipError_t noise_tile(pico_op_t op, int K, const pico_accum_t* acc, uint64_t seed, uint64_t first, int dist,
                      const uint64_t* tp, hipStream_t s) {
  hipError_t e;
  if (op->cs) {
    if ((e = cs_tangents(op, K, nullptr, seed, first, dist, s, tp)) != hipSuccess) return e;
    return timed(op, PICO_PROF_ACCUM, s, [&] {
      return pico::launch_accum_abs2(op->x, acc->sum, acc->sum_im, acc->sumsq, K, (long)op->image(), s);
    });
  }
  if ((e = apply_sigma(op, K, pico::C1_FIRST_PROBE, seed, first, dist, s, tp)) != hipSuccess) return e;
  return accumulate(op, K, acc, seed, first, dist, 0, s, tp);
}

// The same tile replayed from a graph captured (on the operator's own stream,
// which is never run) the first time this (K, dist, accumulator) is seen.
hipError_t noise_tile_graph(pico_op_t op, int K, const pico_accum_t* acc, uint64_t seed, uint64_t first, int dist,
                            hipStream_t s) {
  pico_op_s::TileGraph* g = nullptr;
  for (auto& t : op->graphs)
    if (t.K == K && t.dist == dist && t.sum == acc->sum && t.sum_im == acc->sum_im && t.sumsq == acc->sumsq) g = &t;
  hipError_t e;
  if (!g) {
    if (!op->cap_stream && (e = hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return e;
    if ((e = hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t ec = noise_tile(op, K, acc, 0, 0, dist, op->tile_par, op->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(op->cap_stream, &graph);
    if (ec != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return ec != hipSuccess ? ec : ee;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return e;
    if (op->graphs.size() >= 8) {
      auto lru = std::min_element(op->graphs.begin(), op->graphs.end(),
                                  [](const auto& a, const auto& b) { return a.used < b.used; });
      (void)hipGraphExecDestroy(lru->exec);
      op->graphs.erase(lru);
    }
    op->graphs.push_back({K, dist, acc->sum, acc->sum_im, acc->sumsq, exec, 0});
    g = &op->graphs.back();
  }
  g->used = ++op->graph_clock;
  if ((e = pico::launch_set_tile(op->tile_par, seed, first, s)) != hipSuccess) return e;
  return hipGraphLaunch(g->exec, s);
}

bool kb_grid_dims(const pico_op_desc_t* d, int G[2]);

bool wants_gram(const pico_op_desc_t* d) {
  if (d->sampling != PICO_CART_1D || !pico::gram_supported(d->ny)) return false;
  return d->normal_form == 2;
}

bool wants_gram16(const pico_op_desc_t* d) {
  if (d->sampling != PICO_CART_1D || !pico::gram_supported(d->ny)) return false;
  return d->normal_form == 3;
}

// Kaiser-Bessel tables of a non-Cartesian operator: device buffers in the
// kb_layout order, samples sorted into grid-tile bins on the host
hipError_t build_kb(pico_op_t op, const pico_op_desc_t* d, hipStream_t s) {
  int G[2];
  kb_grid_dims(d, G);
  pico::KbOp& o = op->kb;
  o.M = d->nsamples;
  o.W = d->kb_width;
  o.ny = op->ny;
  o.nx = op->nx;
  o.Gy = G[0];
  o.Gx = G[1];
  o.nby = o.Gy / pico::kKbTile;
  o.nbx = o.Gx / pico::kKbTile;
  const bool normal = d->noncart_normal == 1;
  const pico::KbLayout L = pico::kb_layout(o.M, o.W, o.ny, o.nx, o.Gy, o.Gx, op->K, normal);
  hipError_t e;
  char* part[pico::KbLayout::kParts] = {};
  for (int i = 0; i < pico::KbLayout::kParts; ++i)
    if (L.bytes_of(i) && (e = op->alloc(&part[i], L.bytes_of(i))) != hipSuccess) return e;
  o.sky0 = (int*)part[0];
  o.skx0 = (int*)part[1];
  o.swy = (float*)part[2];
  o.swx = (float*)part[3];
  o.perm = (int*)part[4];
  o.bin_ptr = (int*)part[5];
  o.dy = (float*)part[6];
  o.dx = (float*)part[7];
  o.twx = (float2*)part[8];
  o.twy = (float2*)part[9];
  o.grid = (float2*)part[10];
  o.grid2 = (float2*)part[11];
  const int nslots = (o.Gy / pico::kKbStencilTile) * (o.Gx / pico::kKbStencilTile);
  o.tile_list = normal ? (int*)part[12] : nullptr;
  o.stencil = normal ? (float*)(part[12] + pico::OffsetArena::round_up((size_t)nslots * 4)) : nullptr;
  std::vector<float> traj((size_t)2 * o.M);
  if ((e = hipMemcpyAsync(traj.data(), d->traj, traj.size() * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  std::vector<int> sky0, skx0, perm, bin_ptr;
  std::vector<float> swy, swx, dy, dx;
  pico::kb_build_host(traj.data(), o.M, o.W, d->oversamp, o.ny, o.nx, o.Gy, o.Gx, sky0, skx0, swy, swx, perm,
                      bin_ptr, dy, dx);
  const std::vector<float2> tx = twiddle_table(o.Gx), ty = twiddle_table(o.Gy);
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  if ((e = up(o.sky0, sky0.data(), sky0.size() * 4)) != hipSuccess || (e = up(o.skx0, skx0.data(), skx0.size() * 4)) != hipSuccess ||
      (e = up(o.swy, swy.data(), swy.size() * 4)) != hipSuccess || (e = up(o.swx, swx.data(), swx.size() * 4)) != hipSuccess ||
      (e = up(o.perm, perm.data(), perm.size() * 4)) != hipSuccess ||
      (e = up(o.bin_ptr, bin_ptr.data(), bin_ptr.size() * 4)) != hipSuccess ||
      (e = up(o.dy, dy.data(), dy.size() * 4)) != hipSuccess || (e = up(o.dx, dx.data(), dx.size() * 4)) != hipSuccess ||
      (e = up(o.twx, tx.data(), tx.size() * 8)) != hipSuccess || (e = up(o.twy, ty.data(), ty.size() * 8)) != hipSuccess)
    return e;
  std::vector<int> tile_list;
  std::vector<float> stencil;
  if (normal) {
    pico::kb_build_stencil(sky0, skx0, swy, swx, o.M, o.W, o.Gy, o.Gx, tile_list, o.n_active, stencil);
    if ((e = up(o.tile_list, tile_list.data(), tile_list.size() * 4)) != hipSuccess ||
        (e = up(o.stencil, stencil.data(), stencil.size() * 4)) != hipSuccess)
      return e;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;   // host vectors go out of scope
  op->has_kb = true;
  return hipSuccess;
}

// gridding grid size [Gy, Gx] = oversamp * [ny, nx]; false unless both are integers > n
bool kb_grid_dims(const pico_op_desc_t* d, int G[2]) {
  if (!(d->oversamp > 1.0) || !(d->oversamp <= 4.0)) return false;
  const int n[2] = {d->ny, d->nx};
  for (int i = 0; i < 2; ++i) {
    const double g = d->oversamp * n[i];
    const long r = std::lround(g);
    if (std::fabs(g - (double)r) > 1e-9 || r <= n[i]) return false;
    G[i] = (int)r;
  }
  return true;
}

pico_status_t validate(const pico_op_desc_t* d) {
  if (d->recon != PICO_CGSENSE && d->recon != PICO_CS_FISTA_L1WAV && d->recon != PICO_CS_FISTA_TV)
    return fail(PICO_EUNSUPPORTED, "unknown reconstruction kind");
  if (d->recon == PICO_CS_FISTA_L1WAV || d->recon == PICO_CS_FISTA_TV) {
    if (d->sampling != PICO_CART_2D)
      return fail(PICO_EUNSUPPORTED, "compressed sensing is built for 2-D Cartesian masks");
    if (!d->kdata) return fail(PICO_EINVAL, "compressed sensing needs kdata");
    if (d->fista_iters < 1 || d->fista_iters > 100000) return fail(PICO_EINVAL, "fista_iters must be in 1..100000");
    if (!(d->cs_lambda >= 0.0) || !std::isfinite(d->cs_lambda)) return fail(PICO_EINVAL, "cs_lambda must be finite and >= 0");
    if (d->recon == PICO_CS_FISTA_L1WAV) {
      if (d->wavelet_levels < 1 || d->wavelet_levels > 8) return fail(PICO_EINVAL, "wavelet_levels must be in 1..8");
      const int m = 1 << d->wavelet_levels;
      if (d->ny % m || d->nx % m) return fail(PICO_EINVAL, "ny and nx must be divisible by 2^wavelet_levels");
    } else if (d->tv_inner_iters < 1 || d->tv_inner_iters > 1000) {
      return fail(PICO_EINVAL, "tv_inner_iters must be in 1..1000");
    } else if (d->ny < 14 || d->nx < 38) {
      return fail(PICO_EINVAL, "TV needs ny >= 14 and nx >= 38 (the tangent's tile halos)");
    }
    if (d->power_iters < 1 || !(d->power_margin > 0.0)) return fail(PICO_EINVAL, "compressed sensing needs power_iters >= 1 and power_margin > 0");
  }
  if (d->sampling != PICO_CART_1D && d->sampling != PICO_CART_2D && d->sampling != PICO_NONCART)
    return fail(PICO_EUNSUPPORTED, "unknown sampling kind");
  if (d->ncoils < 1 || d->ncoils > 64) return fail(PICO_EINVAL, "ncoils must be in 1..64");
  if (d->storage != PICO_FP32 && d->storage != PICO_BF16_MAPS && d->storage != PICO_BF16_STREAM)
    return fail(PICO_EINVAL, "unknown storage kind");
  if (d->nx < 2 || d->ny < 2 || (d->ny & 1) || (d->nx & 1)) return fail(PICO_EINVAL, "ny and nx must be even and >= 2");
  if ((int64_t)d->ny * d->nx >= (int64_t)1 << 31) return fail(PICO_EINVAL, "image too large");
  if (d->sampling == PICO_CART_1D) {
    if (!pico::cart1d_supported(d->ny))
      return fail(PICO_EINVAL, "ny=" + std::to_string(d->ny) +
                                   " has no built column FFT (64 96 128 160 192 256 288 320 384 512)");
  } else if (!(d->sampling == PICO_NONCART && d->noncart_normal == 1)) {
    const int f = d->sampling == PICO_NONCART ? 2 : 1;
    if (!pico::grid_line_supported(f * d->ny) || !pico::grid_line_supported(f * d->nx))
      return fail(PICO_EINVAL, "grid " + std::to_string(f * d->ny) + "x" + std::to_string(f * d->nx) +
                                   " has no built FFT length (64 96 128 160 192 256 288 320 384 512 576 640 768)");
    if (pico::grid_cols_lds_bytes(f * d->ny, d->ny) > 160 * 1024)
      return fail(PICO_EINVAL, "column pass does not fit the 160 KiB LDS");
  }
  if (d->cg_iters < 1) return fail(PICO_EINVAL, "cg_iters must be >= 1");
  if (d->probe_tile < 1 || d->probe_tile > 65535) return fail(PICO_EINVAL, "probe_tile must be in 1..65535");
  if (!(d->lambda >= 0.0) || !std::isfinite(d->lambda)) return fail(PICO_EINVAL, "lambda must be finite and >= 0");
  if (!(d->cg_tol >= 0.0)) return fail(PICO_EINVAL, "cg_tol must be >= 0");
  if (!d->maps) return fail(PICO_EINVAL, "maps are required");
  if (d->sampling != PICO_NONCART && !d->mask) return fail(PICO_EINVAL, "mask is required for Cartesian sampling");
  if (d->sampling == PICO_NONCART && (!d->traj || d->nsamples < 1 || d->nsamples > ((int64_t)1 << 30)))
    return fail(PICO_EINVAL, "traj and 1 <= nsamples <= 2^30 are required for non-Cartesian sampling");
  if (d->lambda > 0.0 && (d->power_iters < 1 || !(d->power_margin > 0.0)))
    return fail(PICO_EINVAL, "lambda > 0 needs power_iters >= 1 and power_margin > 0");
  if (d->normal_form < 0 || d->normal_form > 3) return fail(PICO_EINVAL, "normal_form must be 0, 1, 2 or 3");
  if (d->graph != 0 && d->graph != 1) return fail(PICO_EINVAL, "graph must be 0 or 1");
  if (d->noncart_normal != 0 && d->noncart_normal != 1) return fail(PICO_EINVAL, "noncart_normal must be 0 or 1");
  if (d->noncart_normal == 1 && (d->sampling != PICO_NONCART || d->kb_width == 0))
    return fail(PICO_EINVAL, "the gridding normal operator needs PICO_NONCART and kb_width > 0");
  if (d->normal_form >= 2 && (d->sampling != PICO_CART_1D || !pico::gram_supported(d->ny)))
    return fail(PICO_EINVAL, "the dense normal form needs PICO_CART_1D and ny a multiple of 32 in 64..512");
  if (d->kb_width != 0) {
    if (d->sampling != PICO_NONCART) return fail(PICO_EINVAL, "kb_width applies to PICO_NONCART only");
    if (d->kb_width < 2 || d->kb_width > 8 || (d->kb_width & 1))
      return fail(PICO_EINVAL, "kb_width must be even in 2..8");
    int G[2];
    if (!kb_grid_dims(d, G)) return fail(PICO_EINVAL, "oversamp * ny and oversamp * nx must be integers > n");
    if (G[0] % pico::kKbTile || G[1] % pico::kKbTile)
      return fail(PICO_EINVAL, "the gridding grid must be a multiple of 16 points per axis");
    for (int g : G)
      if (!pico::grid_line_supported(g))
        return fail(PICO_EINVAL, "gridding length " + std::to_string(g) +
                                     " has no built FFT length (64 96 128 160 192 256 288 320 384 512 576 640 768)");
    if (pico::grid_cols_lds_bytes(G[0], G[0]) > 160 * 1024)
      return fail(PICO_EINVAL, "gridding column pass does not fit the 160 KiB LDS");
    if ((double)d->nsamples * d->kb_width * d->kb_width >= 2147483647.0)
      return fail(PICO_EINVAL, "nsamples * kb_width^2 must stay below 2^31");
  }
  return PICO_OK;
}

}  // namespace

extern "C" {

const char* pico_last_error(void) { return g_err.c_str(); }

pico_status_t pico_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* ptr, void* ctx),
                                 void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(PICO_EINVAL, "pico_set_allocator needs both callbacks, or neither to restore hipMalloc / hipFree");
  std::lock_guard<std::mutex> lk(pico::g_alloc_mu);
  pico::g_alloc.alloc = alloc;
  pico::g_alloc.free = free_fn;
  pico::g_alloc.ctx = alloc ? ctx : nullptr;
  return PICO_OK;
}

}  // extern "C"

namespace pico {

pico_status_t set_error(pico_status_t st, const std::string& msg) { return fail(st, msg); }

// Device bytes pico_init takes for d: resident after it returns, and the peak
// during it (temporaries of the weight builders and of the CS primal).  Each
// allocation is counted in 256-byte pieces, in the order pico_init makes it.
pico_status_t estimate_bytes(const pico_op_desc_t* d, size_t* resident, size_t* peak) {
  if (!d) return fail(PICO_EINVAL, "NULL descriptor");
  if (pico_status_t st = validate(d)) return st;
  size_t cur = 0, top = 0;
  auto add = [&](size_t b) {
    cur += OffsetArena::round_up(b);
    top = std::max(top, cur);
  };
  auto sub = [&](size_t b) { cur -= OffsetArena::round_up(b); };
  const size_t nc = d->ncoils, ny = d->ny, nx = d->nx, n = ny * nx, K = d->probe_tile;
  const bool colmajor = d->sampling == PICO_CART_1D;
  const size_t f = d->sampling == PICO_NONCART ? 2 : 1, Gy = f * ny, Gx = f * nx;
  const size_t nblk = colmajor ? nx : ny;
  add(n * nc * 8);
  if (d->storage != PICO_FP32) add(n * nc * 4);
  for (int i = 0; i < 4; ++i) add(n * K * 8);
  add(K * nblk * 4 * 8);
  add(512 * 8);
  for (int i = 0; i < 4; ++i) add(K * 8);
  add(K * 4);
  if (d->graph) add(2 * 8);
  const size_t linv = 2 * nc * nc * 8;
  add(linv);
  if (colmajor) {
    add(ny * 4);
    add(ny * 8);
    if (wants_gram(d)) {
      add(gram_bytes(d->ny, d->nx));
      add(ny * 16);
    }
    if (wants_gram16(d)) {
      add(gram_bytes(d->ny, d->nx));
      add(ny * 16);
      add(d->nx * 4);
      add(pico::gram16_pexp_count(d->nx, K) * 4);
    }
  } else {
    const bool kbn = d->noncart_normal == 1;
    if (!kbn) {
      add(Gy * Gx * 4);
      add(Gx * 8);
      add(Gy * 8);
      add(K * nc * ny * Gx * 8);
    }
    if (d->sampling == PICO_NONCART) {
      if (!kbn) {
        const size_t sc = toeplitz_scratch_bytes(d->nsamples, d->ny, d->nx);
        add(sc);
        sub(sc);
      }
      if (d->kb_width > 0) {
        int G[2];
        kb_grid_dims(d, G);
        const KbLayout L = kb_layout(d->nsamples, d->kb_width, d->ny, d->nx, G[0], G[1], d->probe_tile, kbn);
        for (int i = 0; i < KbLayout::kParts; ++i)
          if (L.bytes_of(i)) add(L.bytes_of(i));
      }
    }
  }
  if (d->sampling == PICO_CART_2D) add(n);
  if (d->recon == PICO_CS_FISTA_L1WAV || d->recon == PICO_CS_FISTA_TV) {
    const bool tv = d->recon == PICO_CS_FISTA_TV;
    add(n * K * 8);
    if (tv) {
      for (int i = 0; i < 4; ++i) add(2 * n * K * 8);
      add(n * (size_t)d->fista_iters * d->tv_inner_iters * 16);
      add(n * (size_t)d->fista_iters * d->tv_inner_iters * 4);
    } else {
      add(n * K * 8);
      add(n * (size_t)d->fista_iters * 16);
    }
    add(n * 8);
    add(nc * n * 16);   // FP64 maps, DFT matrices, A^H b, x_T (resident)
    add(ny * ny * 16);
    add(nx * nx * 16);
    add(n * 16);
    add(n * 16);
    const size_t tmp[] = {nc * n * 16, nc * n * 16, n * 16, n * 16, n * 16, n * 16, 2 * CS64_DOT_BLOCKS * 8,
                          tv ? 2 * n * 16 : 0, tv ? 2 * n * 16 : 0, tv ? n * 16 : 0};
    for (size_t b : tmp) if (b) add(b);
    for (size_t b : tmp) if (b) sub(b);
  }
  sub(linv);
  if (resident) *resident = cur;
  if (peak) *peak = top;
  return PICO_OK;
}

pico_status_t init_in_arena(const pico_op_desc_t* d, void* stream, DeviceArena* arena, pico_op_t* out);

}  // namespace pico

extern "C" {

pico_status_t pico_estimate_bytes(const pico_op_desc_t* d, uint64_t* resident, uint64_t* peak) {
  size_t r = 0, p = 0;
  if (pico_status_t st = pico::estimate_bytes(d, &r, &p)) return st;
  if (resident) *resident = r;
  if (peak) *peak = p;
  return PICO_OK;
}

pico_status_t pico_op_bytes(pico_op_t op, uint64_t* resident, uint64_t* peak) {
  if (!op) return fail(PICO_EINVAL, "NULL handle");
  if (resident) *resident = op->bytes;
  if (peak) *peak = op->peak;
  return PICO_OK;
}

pico_status_t pico_init(const pico_op_desc_t* d, void* stream, pico_op_t* out) {
  return pico::init_in_arena(d, stream, nullptr, out);
}

}  // extern "C"

pico_status_t pico::init_in_arena(const pico_op_desc_t* d, void* stream, pico::DeviceArena* arena,
                                  pico_op_t* out) {
  if (!d || !out) return fail(PICO_EINVAL, "NULL descriptor or output handle");
  *out = nullptr;
  if (pico_status_t st = validate(d)) return st;
  hipStream_t s = (hipStream_t)stream;
  const int nc = d->ncoils, ny = d->ny, nx = d->nx;
  std::vector<double> linv;
  if (d->psi) {
    std::string why;
    if (!cholesky_inverse(d->psi, nc, linv, why)) return fail(PICO_EINVAL, why);
  } else {
    linv.assign(2 * nc * nc, 0.0);
    for (int c = 0; c < nc; ++c) linv[2 * (c * nc + c)] = 1.0;
  }

  auto* op = new pico_op_s();
  op->arena = arena;
  op->ny = ny;
  op->nx = nx;
  op->nc = nc;
  op->sampling = d->sampling;
  op->recon = d->recon;
  op->cg_iters = d->cg_iters;
  op->cg_tol = d->cg_tol;
  op->lam_rel = d->lambda;
  op->K = d->probe_tile;
  op->last_stream = s;
  op->colmajor = d->sampling == PICO_CART_1D;
  op->nblk = op->colmajor ? nx : ny;
  if (!op->colmajor) {
    const int f = d->sampling == PICO_NONCART ? 2 : 1;
    op->Gy = f * ny;
    op->Gx = f * nx;
  }
  const size_t n = op->image();
  const int K = op->K;

  double* linv_d = nullptr;
  hipError_t e = hipSuccess;
  auto bad = [&](hipError_t err, const char* what) {
    delete op;
    if (err == hipErrorOutOfMemory || err == hipErrorMemoryAllocation)
      return fail(PICO_ENOMEM, std::string(what) + ": out of device memory");
    return fail(PICO_EDEVICE, std::string(what) + ": " + hipGetErrorString(err));
  };
  if ((e = op->alloc(&op->maps, n * nc)) != hipSuccess) return bad(e, "maps");
  if (d->storage != PICO_FP32 && (e = op->alloc(&op->maps_bf, n * nc)) != hipSuccess) return bad(e, "bfloat16 maps");
  op->stream_bf = d->storage == PICO_BF16_STREAM && d->sampling != PICO_CART_1D;
  if ((e = op->alloc(&op->x, n * K)) != hipSuccess) return bad(e, "workspace x");
  if ((e = op->alloc(&op->r, n * K)) != hipSuccess) return bad(e, "workspace r");
  if ((e = op->alloc(&op->p, n * K)) != hipSuccess) return bad(e, "workspace p");
  if ((e = op->alloc(&op->q, n * K)) != hipSuccess) return bad(e, "workspace q");
  if ((e = op->alloc(&op->part, (size_t)K * op->nblk * 4)) != hipSuccess) return bad(e, "partials");
  if ((e = op->alloc(&op->mon, 512)) != hipSuccess) return bad(e, "monitor");
  if ((e = op->alloc(&op->alpha, K)) != hipSuccess) return bad(e, "scalars");
  if ((e = op->alloc(&op->beta, K)) != hipSuccess) return bad(e, "scalars");
  if ((e = op->alloc(&op->rr, K)) != hipSuccess) return bad(e, "scalars");
  if ((e = op->alloc(&op->rr0, K)) != hipSuccess) return bad(e, "scalars");
  if ((e = op->alloc(&op->state, K)) != hipSuccess) return bad(e, "scalars");
  op->use_graph = d->graph != 0;
  if (op->use_graph && (e = op->alloc(&op->tile_par, 2)) != hipSuccess) return bad(e, "tile parameters");
  if ((e = op->alloc(&linv_d, linv.size())) != hipSuccess) return bad(e, "whitening");
  if ((e = hipMemcpyAsync(linv_d, linv.data(), linv.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess) return bad(e, "upload");

  if (op->colmajor) {
    // sampling weights: the centred DFT is (-1)^(ny/2) D F D with D = (-1)^y,
    // so the centred-order mask applies unchanged to the plain FFT output;
    // w[k] = mask[k] / ny carries the orthonormal scaling of F^H P F.
    if ((e = op->alloc(&op->maskw, ny)) != hipSuccess) return bad(e, "mask");
    if ((e = op->alloc(&op->twt, ny)) != hipSuccess) return bad(e, "twiddles");
    std::vector<uint8_t> mask_h(ny);
    if ((e = hipMemcpyAsync(mask_h.data(), d->mask, ny, hipMemcpyDeviceToHost, s)) != hipSuccess) return bad(e, "mask copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "mask copy");
    std::vector<float> w(ny);
    for (int k = 0; k < ny; ++k) w[k] = mask_h[k] ? (float)(1.0 / ny) : 0.0f;
    std::vector<float2> tw = twiddle_table(ny);
    if ((e = hipMemcpyAsync(op->maskw, w.data(), ny * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess) return bad(e, "upload");
    if ((e = hipMemcpyAsync(op->twt, tw.data(), ny * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess) return bad(e, "upload");
    if ((e = pico::launch_prep_maps_cart1d((const float2*)d->maps, linv_d, op->maps, nc, ny, nx, s)) != hipSuccess) return bad(e, "prep maps");
    if (op->maps_bf && (e = pico::launch_quantise_maps(op->maps, op->maps_bf, (long)(n * nc), true, s)) != hipSuccess) return bad(e, "bfloat16 maps");
    if (wants_gram(d)) {
      if ((e = op->alloc(&op->gram, pico::gram_bytes(ny, nx) / sizeof(float2))) != hipSuccess) return bad(e, "dense blocks");
      if ((e = op->alloc(&op->gram_c, ny)) != hipSuccess) return bad(e, "dense blocks");
      if ((e = pico::build_gram(op->maps, w.data(), nc, ny, nx, op->gram, op->gram_c, s)) != hipSuccess) return bad(e, "dense blocks");
      op->use_gram = true;
    }
    if (wants_gram16(d)) {
      if ((e = op->alloc(&op->gram16, pico::gram_bytes(ny, nx) / sizeof(uint32_t))) != hipSuccess) return bad(e, "dense blocks");
      if ((e = op->alloc(&op->gram_c, ny)) != hipSuccess) return bad(e, "dense blocks");
      if ((e = op->alloc(&op->gram16_exp, nx)) != hipSuccess) return bad(e, "dense blocks");
      if ((e = op->alloc(&op->gram16_pexp, pico::gram16_pexp_count(nx, op->K))) != hipSuccess) return bad(e, "dense blocks");
      if ((e = pico::build_gram16(op->maps, w.data(), nc, ny, nx, op->gram16, op->gram16_exp, op->gram_c, s)) != hipSuccess)
        return bad(e, "dense blocks");
      op->use_gram16 = true;
    }
  } else {
    const int Gy = op->Gy, Gx = op->Gx;
    // the gridding normal operator works on the Kaiser-Bessel grid alone: no
    // Toeplitz weights, no row-transformed planes
    op->kb_normal = d->noncart_normal == 1;
    std::vector<float2> tx = twiddle_table(Gx), ty = twiddle_table(Gy);
    if (!op->kb_normal) {
      if ((e = op->alloc(&op->w, (size_t)Gy * Gx)) != hipSuccess) return bad(e, "weights");
      if ((e = op->alloc(&op->twx, Gx)) != hipSuccess) return bad(e, "twiddles");
      if ((e = op->alloc(&op->twy, Gy)) != hipSuccess) return bad(e, "twiddles");
      if ((e = op->alloc(&op->T, (size_t)K * nc * ny * Gx)) != hipSuccess) return bad(e, "grid workspace");
      if ((e = hipMemcpyAsync(op->twx, tx.data(), Gx * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess) return bad(e, "upload");
      if ((e = hipMemcpyAsync(op->twy, ty.data(), Gy * sizeof(float2), hipMemcpyHostToDevice, s)) != hipSuccess) return bad(e, "upload");
    }
    const int fold = d->sampling == PICO_CART_2D;
    if ((e = pico::launch_prep_maps_rowmajor((const float2*)d->maps, linv_d, op->maps, nc, ny, nx, fold, s)) != hipSuccess) return bad(e, "prep maps");
    // CG-SENSE: the rounded maps define the operator on every path (the FP32
    // copy is rounded too).  Compressed sensing: bfloat16 is a storage form of
    // the normal-operator reads in the tangents only; the FP64 primal (the
    // linearisation point and its active set) and the k-space adjoint of the
    // probes keep the unrounded maps.
    if (op->maps_bf && (e = pico::launch_quantise_maps(op->maps, op->maps_bf, (long)(n * nc), d->recon == PICO_CGSENSE, s)) != hipSuccess) return bad(e, "bfloat16 maps");
    if (d->sampling == PICO_CART_2D) {
      if ((e = pico::launch_mask_weights(d->mask, op->w, ny, nx, (float)(1.0 / ((double)ny * nx)), s)) != hipSuccess) return bad(e, "weights");
    } else {
      if (!op->kb_normal) {
        char* tscratch = nullptr;
        if ((e = op->alloc(&tscratch, pico::toeplitz_scratch_bytes(d->nsamples, ny, nx))) != hipSuccess) return bad(e, "Toeplitz scratch");
        if ((e = pico::build_toeplitz_weights(d->traj, d->nsamples, ny, nx, op->w, tscratch, s)) != hipSuccess) return bad(e, "Toeplitz weights");
        op->release(tscratch);
      }
      if (d->kb_width > 0) {
        if ((e = build_kb(op, d, s)) != hipSuccess) return bad(e, "gridding tables");
      }
    }
  }

  // spectral normalisation (Sec. 3.2.1, 3.3): lambda_max of M by power steps
  // (the compressed-sensing operator takes it from its FP64 primal below)
  if (d->lambda > 0.0 && d->recon == PICO_CGSENSE) {
    double lam_hat = 0.0;
    if ((e = power_lambda(op, d->power_iters, &lam_hat, s)) != hipSuccess) return bad(e, "power");
    op->s2 = d->power_margin * lam_hat;
    op->lam_abs = d->lambda * op->s2;
  }
  if (d->sampling == PICO_CART_2D) {
    if ((e = op->alloc(&op->mask_d, n)) != hipSuccess) return bad(e, "mask");
    if ((e = hipMemcpyAsync(op->mask_d, d->mask, n, hipMemcpyDeviceToDevice, s)) != hipSuccess) return bad(e, "mask copy");
  }
  if (d->recon == PICO_CS_FISTA_L1WAV || d->recon == PICO_CS_FISTA_TV) {
    // FISTA primal at the measured data in FP64, storing the trajectory the
    // tangents need: c_k = Psi z_k, or the TV projection data of every inner
    // step (Sec. 2.2 CS extension, Sec. 3.2.3, 3.3)
    const bool tv = d->recon == PICO_CS_FISTA_TV;
    op->cs = true;
    op->fista_T = d->fista_iters;
    op->levels = tv ? 0 : d->wavelet_levels;
    op->tv_inner = tv ? d->tv_inner_iters : 0;
    op->cs_lam = d->cs_lambda;
    auto momentum = [](int count, std::vector<double>& w64, std::vector<float>& w32) {
      double t = 1.0;
      for (int k = 0; k < count; ++k) {
        const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
        w64.push_back((t - 1.0) / tn);
        w32.push_back((float)w64.back());
        t = tn;
      }
    };
    momentum(op->fista_T, op->theta64, op->theta);
    momentum(op->tv_inner, op->tv_th64, op->tv_th);
    if ((e = op->alloc(&op->wA, n * K)) != hipSuccess) return bad(e, "tangent buffer");
    if (tv) {
      const size_t steps = (size_t)op->fista_T * op->tv_inner;
      if ((e = op->alloc(&op->tv_dp, 2 * n * K)) != hipSuccess || (e = op->alloc(&op->tv_dpB, 2 * n * K)) != hipSuccess ||
          (e = op->alloc(&op->tv_drA, 2 * n * K)) != hipSuccess || (e = op->alloc(&op->tv_drB, 2 * n * K)) != hipSuccess)
        return bad(e, "TV dual tangents");
      if ((e = op->alloc(&op->tv_what, n * steps)) != hipSuccess || (e = op->alloc(&op->tv_invn, n * steps)) != hipSuccess)
        return bad(e, "TV projection data");
    } else {
      if ((e = op->alloc(&op->wB, n * K)) != hipSuccess) return bad(e, "wavelet buffer");
      if ((e = op->alloc(&op->ctraj, n * (size_t)op->fista_T)) != hipSuccess) return bad(e, "FISTA trajectory");
    }
    if ((e = op->alloc(&op->xrec, n)) != hipSuccess) return bad(e, "reconstruction");
    // resident FP64 operator (whitened maps, centred DFT matrices), A^H b and
    // x_T: the linearisation point, kept for the replicas of pico_pmr_cs
    pico::Cs64& o = op->c64;
    o.ny = ny;
    o.nx = nx;
    o.nc = nc;
    o.levels = op->levels;
    o.mask = op->mask_d;
    o.ctraj = op->ctraj;
    o.tv_inner = op->tv_inner;
    o.tv_th = op->tv_th64.data();
    o.tv_what = op->tv_what;
    o.tv_invn = op->tv_invn;
    if ((e = op->alloc(&o.S, (size_t)nc * n)) != hipSuccess || (e = op->alloc(&o.Fy, (size_t)ny * ny)) != hipSuccess ||
        (e = op->alloc(&o.Fx, (size_t)nx * nx)) != hipSuccess || (e = op->alloc(&op->atb64, n)) != hipSuccess ||
        (e = op->alloc(&op->x64, n)) != hipSuccess)
      return bad(e, "FP64 operator");
    double2 *y = nullptr, *z = nullptr, *tmp = nullptr, *q = nullptr;
    double* part = nullptr;
    if ((e = op->alloc(&o.U, (size_t)nc * n)) != hipSuccess || (e = op->alloc(&o.V, (size_t)nc * n)) != hipSuccess ||
        (e = op->alloc(&y, n)) != hipSuccess || (e = op->alloc(&z, n)) != hipSuccess ||
        (e = op->alloc(&tmp, n)) != hipSuccess || (e = op->alloc(&q, n)) != hipSuccess ||
        (e = op->alloc(&part, 2 * pico::CS64_DOT_BLOCKS)) != hipSuccess)
      return bad(e, "FP64 primal workspace");
    if (tv && ((e = op->alloc(&o.tv_r, 2 * n)) != hipSuccess || (e = op->alloc(&o.tv_p, 2 * n)) != hipSuccess ||
               (e = op->alloc(&o.tv_u, n)) != hipSuccess))
      return bad(e, "FP64 TV workspace");
    if ((e = pico::cs64_setup(o, (const float2*)d->maps, linv_d, s)) != hipSuccess) return bad(e, "FP64 primal");
    double lam_hat = 0.0;
    if ((e = pico::cs64_power(o, d->power_iters, y, z, part, &lam_hat, s)) != hipSuccess) return bad(e, "power");
    op->s2 = d->power_margin * lam_hat;
    if ((e = pico::cs64_adjoint_kdata(o, (const float2*)d->kdata, linv_d, op->atb64, s)) != hipSuccess) return bad(e, "A^H b");
    if ((e = pico::cs64_fista(o, 1, op->atb64, op->s2, op->cs_lam, op->fista_T, op->theta64.data(), true, y,
                              op->x64, z, tmp, q, s)) != hipSuccess)
      return bad(e, "FISTA");
    if ((e = pico::launch_to_f32(op->x64, op->xrec, (long)n, s)) != hipSuccess) return bad(e, "reconstruction");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "FISTA");
    for (void* ptr : {(void*)o.U, (void*)o.V, (void*)y, (void*)z, (void*)tmp, (void*)q, (void*)part, (void*)o.tv_r,
                      (void*)o.tv_p, (void*)o.tv_u})
      if (ptr) op->release(ptr);
    o.U = o.V = nullptr;
    o.tv_r = o.tv_p = o.tv_u = nullptr;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "init");
  op->release(linv_d);
  *out = op;
  return PICO_OK;
}

extern "C" {

double pico_lambda_abs(pico_op_t op) { return op ? op->lam_abs : NAN; }

pico_status_t pico_apply_jvp(pico_op_t op, const void* w, void* u, int32_t k, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!op->cs) return fail(PICO_EUNSUPPORTED, "pico_apply_jvp needs a compressed-sensing operator");
  if (!w || !u) return fail(PICO_EINVAL, "NULL w or u");
  if (k < 1 || k > op->K) return fail(PICO_EINVAL, "k must be in 1..probe_tile");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  HIP_OR_RETURN(cs_tangents(op, k, (const float2*)w, 0, 0, 0, s));
  HIP_OR_RETURN(hipMemcpyAsync(u, op->x, (size_t)k * op->image() * sizeof(float2), hipMemcpyDeviceToDevice, s));
  return PICO_OK;
}

pico_status_t pico_recon(pico_op_t op, void* x, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!op->cs) return fail(PICO_EUNSUPPORTED, "the reconstruction is kept for compressed-sensing operators");
  if (!x) return fail(PICO_EINVAL, "NULL output");
  HIP_OR_RETURN(hipMemcpyAsync(x, op->xrec, op->image() * sizeof(float2), hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
  return PICO_OK;
}

pico_status_t pico_apply_nufft(pico_op_t op, int32_t adjoint, const void* in, void* out, int32_t k,
                               void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!op->has_kb) return fail(PICO_EUNSUPPORTED, "the operator has no gridding data path (PICO_NONCART, kb_width > 0)");
  if (!in || !out) return fail(PICO_EINVAL, "NULL input or output");
  if (k < 1 || k > op->K) return fail(PICO_EINVAL, "k must be in 1..probe_tile");
  if (adjoint != 0 && adjoint != 1) return fail(PICO_EINVAL, "adjoint must be 0 or 1");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  if (adjoint) HIP_OR_RETURN(pico::kb_adjoint(op->kb, op->maps, op->nc, k, (const float2*)in, 0, 0, (float2*)out, s));
  else HIP_OR_RETURN(pico::kb_forward(op->kb, op->maps, op->nc, k, (const float2*)in, (float2*)out, s));
  return PICO_OK;
}

pico_status_t pico_apply_cov(pico_op_t op, const void* v, void* u, int32_t k, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (op->cs) return fail(PICO_EUNSUPPORTED, "a compressed-sensing operator has no linear covariance; use pico_apply_jvp");
  if (!v || !u) return fail(PICO_EINVAL, "NULL v or u");
  if (k < 1 || k > op->K) return fail(PICO_EINVAL, "k must be in 1..probe_tile");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  const size_t bytes = (size_t)k * op->image() * sizeof(float2);
  if (op->colmajor) HIP_OR_RETURN(pico::launch_transpose_in((const float2*)v, op->r, k, op->ny, op->nx, s));
  else HIP_OR_RETURN(hipMemcpyAsync(op->r, v, bytes, hipMemcpyDeviceToDevice, s));
  HIP_OR_RETURN(apply_sigma(op, k, pico::C1_FIRST_BUF, 0, 0, 0, s));
  if (op->colmajor) HIP_OR_RETURN(pico::launch_transpose_out(op->x, (float2*)u, k, op->ny, op->nx, s));
  else HIP_OR_RETURN(hipMemcpyAsync(u, op->x, bytes, hipMemcpyDeviceToDevice, s));
  return PICO_OK;
}

pico_status_t pico_noise_map(pico_op_t op, uint64_t seed, int64_t first_probe, int64_t nprobes,
                             int32_t dist, pico_accum_t* acc, pico_stats_t* stats, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum) return fail(PICO_EINVAL, "accumulator with a sum buffer is required");
  if (nprobes < 0 || first_probe < 0) return fail(PICO_EINVAL, "negative probe range");
  if (dist < 0 || dist > 3) return fail(PICO_EINVAL, "unknown probe family");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  const bool graph = op->use_graph && !op->prof_on;
  auto tile = [&](int K, uint64_t first) {
    return graph ? noise_tile_graph(op, K, acc, seed, first, dist, s)
                 : noise_tile(op, K, acc, seed, first, dist, nullptr, s);
  };
  if (op->cs) {
    for (int64_t done = 0; done < nprobes;) {
      const int K = (int)std::min<int64_t>(op->K, nprobes - done);
      HIP_OR_RETURN(tile(K, (uint64_t)(first_probe + done)));
      done += K;
    }
    acc->count += nprobes;
    if (stats) {
      HIP_OR_RETURN(hipStreamSynchronize(s));
      stats->probes = nprobes;
      stats->max_relres = stats->mean_relres = 0.0;
      stats->frozen = 0;
      stats->lambda_abs = 0.0;
    }
    return PICO_OK;
  }
  StatAcc sa;
  for (int64_t done = 0; done < nprobes;) {
    const int K = (int)std::min<int64_t>(op->K, nprobes - done);
    HIP_OR_RETURN(tile(K, (uint64_t)(first_probe + done)));
    if (stats) HIP_OR_RETURN(collect_stats(op, K, s, sa));
    done += K;
  }
  acc->count += nprobes;
  if (stats) return write_stats(op, sa, stats);
  return PICO_OK;
}

pico_status_t pico_finalize(pico_op_t op, const pico_accum_t* acc, double* var, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !var) return fail(PICO_EINVAL, "NULL accumulator or output");
  if (acc->count < 1) return fail(PICO_EINVAL, "no probes accumulated");
  HIP_OR_RETURN(pico::launch_finalize(acc->sum, var, (int64_t)op->image(), 1.0 / (double)acc->count,
                                      (hipStream_t)stream));
  return PICO_OK;
}

pico_status_t pico_pmr_baseline(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep,
                                pico_accum_t* acc, pico_stats_t* stats, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !acc->sum_im || !acc->sumsq)
    return fail(PICO_EINVAL, "PMR needs sum, sum_im and sumsq buffers");
  if (nrep < 0 || first < 0) return fail(PICO_EINVAL, "negative replica range");
  if (op->cs) return fail(PICO_EUNSUPPORTED, "a compressed-sensing operator takes pico_pmr_cs");
  if (op->sampling == PICO_NONCART && !op->has_kb)
    return fail(PICO_EUNSUPPORTED, "PMR on non-Cartesian sampling needs the gridding data path (kb_width > 0)");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  StatAcc sa;
  for (int64_t done = 0; done < nrep;) {
    const int K = (int)std::min<int64_t>(op->K, nrep - done);
    const uint64_t f = (uint64_t)(first + done);
    if (op->colmajor) {
      NormalCall c;
      c.seed = seed;
      c.first = f;
      HIP_OR_RETURN(timed(op, PICO_PROF_OTHER, s, [&] { return launch_normal(op, K, pico::C1_PMR_RHS, c, s); }));
    } else if (op->sampling == PICO_NONCART) {
      // r = A^H n by gridding, CN(0, I) noise on every coil sample (Philox stream 1)
      HIP_OR_RETURN(timed(op, PICO_PROF_OTHER, s, [&] {
        return pico::kb_adjoint(op->kb, op->maps, op->nc, K, nullptr, seed, f, op->r, s);
      }));
    } else {
      // r = A^H n, white Gaussian k-space noise on the mask (Philox stream 1)
      HIP_OR_RETURN(timed(op, PICO_PROF_OTHER, s, [&] {
        return adjoint_kspace(op, K, nullptr, nullptr, seed, f, 1u, 3, op->r, s);
      }));
    }
    HIP_OR_RETURN(cg_solve(op, K, pico::C1_FIRST_BUF, 0, 0, 0, s));
    HIP_OR_RETURN(accumulate(op, K, acc, 0, 0, 0, 1, s));
    if (stats) HIP_OR_RETURN(collect_stats(op, K, s, sa));
    done += K;
  }
  acc->count += nrep;
  if (stats) return write_stats(op, sa, stats);
  return PICO_OK;
}

pico_status_t pico_pmr_cs(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep, double sigma,
                          pico_accum_t* acc, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!op->cs) return fail(PICO_EUNSUPPORTED, "pico_pmr_cs needs a compressed-sensing operator");
  if (!acc || !acc->sum || !acc->sum_im || !acc->sumsq)
    return fail(PICO_EINVAL, "PMR needs sum, sum_im and sumsq buffers");
  if (nrep < 0 || first < 0) return fail(PICO_EINVAL, "negative replica range");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(PICO_EINVAL, "sigma must be finite and > 0");
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  const size_t n = op->image();
  pico::Cs64& o = op->c64;
  if (op->pmr_B == 0) {
    const int B = std::min(op->K, 16);
    hipError_t e;
    const bool tv = op->tv_inner > 0;
    if ((e = op->alloc(&o.U, (size_t)B * op->nc * n)) != hipSuccess || (e = op->alloc(&o.V, (size_t)B * op->nc * n)) != hipSuccess ||
        (e = op->alloc(&op->pmr_atb, B * n)) != hipSuccess || (e = op->alloc(&op->pmr_y, B * n)) != hipSuccess ||
        (e = op->alloc(&op->pmr_x, B * n)) != hipSuccess || (e = op->alloc(&op->pmr_z, B * n)) != hipSuccess ||
        (e = op->alloc(&op->pmr_tmp, B * n)) != hipSuccess || (e = op->alloc(&op->pmr_q, B * n)) != hipSuccess ||
        (tv && ((e = op->alloc(&op->pmr_tv_r, 2 * B * n)) != hipSuccess ||
                (e = op->alloc(&op->pmr_tv_p, 2 * B * n)) != hipSuccess ||
                (e = op->alloc(&op->pmr_tv_u, B * n)) != hipSuccess))) {
      for (void* p : {(void*)o.U, (void*)o.V, (void*)op->pmr_atb, (void*)op->pmr_y, (void*)op->pmr_x,
                      (void*)op->pmr_z, (void*)op->pmr_tmp, (void*)op->pmr_q, (void*)op->pmr_tv_r,
                      (void*)op->pmr_tv_p, (void*)op->pmr_tv_u})
        if (p) op->release(p);
      o.U = o.V = nullptr;
      op->pmr_atb = op->pmr_y = op->pmr_x = op->pmr_z = op->pmr_tmp = op->pmr_q = nullptr;
      op->pmr_tv_r = op->pmr_tv_p = op->pmr_tv_u = nullptr;
      return fail(e == hipErrorOutOfMemory ? PICO_ENOMEM : PICO_EDEVICE, "PMR workspace");
    }
    o.tv_r = op->pmr_tv_r;
    o.tv_p = op->pmr_tv_p;
    o.tv_u = op->pmr_tv_u;
    op->pmr_B = B;
  }
  for (int64_t done = 0; done < nrep;) {
    const int B = (int)std::min<int64_t>(op->pmr_B, nrep - done);
    HIP_OR_RETURN(timed(op, PICO_PROF_OTHER, s, [&] {
      return pico::cs64_pmr(o, B, op->atb64, op->x64, op->s2, op->cs_lam, op->fista_T, op->theta64.data(), seed,
                            (uint64_t)(first + done), sigma, op->pmr_atb, op->pmr_y, op->pmr_x, op->pmr_z,
                            op->pmr_tmp, op->pmr_q, acc->sum, acc->sum_im, acc->sumsq, s);
    }));
    done += B;
  }
  acc->count += nrep;
  return PICO_OK;
}

}  // extern "C"

// Workspace of pico_pmr_cs_noalloc: a fixed device array, one copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static constexpr size_t kNoallocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoallocBytes];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
char* g_scratch_dev[kMaxDevices] = {};   // guarded by g_scratch_mu

// Device address of `scratch` on the current device (looked up on first use)
pico_status_t scratch_address(char** out) {
  int dev = -1;
  HIP_OR_RETURN(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PICO_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIP_OR_RETURN(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PICO_EDEVICE, "no device address for the static workspace");
    g_scratch_dev[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return PICO_OK;
}

}  // namespace

extern "C" {

pico_status_t pico_pmr_cs_noalloc(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep, double sigma,
                                  pico_accum_t* acc, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!op->cs) return fail(PICO_EUNSUPPORTED, "pico_pmr_cs_noalloc needs a compressed-sensing operator");
  if (!acc || !acc->sum || !acc->sum_im || !acc->sumsq)
    return fail(PICO_EINVAL, "PMR needs sum, sum_im and sumsq buffers");
  if (nrep < 0 || first < 0) return fail(PICO_EINVAL, "negative replica range");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(PICO_EINVAL, "sigma must be finite and > 0");
  // the same replica batches as pico_pmr_cs, so the sums agree bit for bit
  const int B = std::min(op->K, 16);
  const size_t n = op->image();
  const bool tv = op->tv_inner > 0;
  const size_t img = pico::OffsetArena::round_up((size_t)B * n * sizeof(double2));
  const size_t coil = pico::OffsetArena::round_up((size_t)B * op->nc * n * sizeof(double2));
  const size_t need = 2 * coil + 6 * img + (tv ? 5 * img : 0);
  if (need > kNoallocBytes)
    return fail(PICO_EINVAL, "replica workspace of " + std::to_string(need) + " bytes (" + std::to_string(B) +
                                 " replicas of " + std::to_string(op->ny) + "x" + std::to_string(op->nx) + "x" +
                                 std::to_string(op->nc) + ") exceeds the static " +
                                 std::to_string(kNoallocBytes >> 20) + " MiB workspace");
  char* base = nullptr;
  if (pico_status_t st = scratch_address(&base)) return st;
  hipStream_t s = (hipStream_t)stream;
  op->last_stream = s;
  // every piece is written before it is read (noise draw, zero starts), so
  // nothing left by an earlier call needs clearing
  pico::Cs64 o = op->c64;
  char* cur = base;
  auto take = [&](size_t bytes) {
    double2* p = reinterpret_cast<double2*>(cur);
    cur += bytes;
    return p;
  };
  o.U = take(coil);
  o.V = take(coil);
  double2 *atb = take(img), *y = take(img), *x = take(img), *z = take(img), *tmp = take(img), *q = take(img);
  if (tv) {
    o.tv_r = take(2 * img);
    o.tv_p = take(2 * img);
    o.tv_u = take(img);
  }
  for (int64_t done = 0; done < nrep;) {
    const int b = (int)std::min<int64_t>(B, nrep - done);
    HIP_OR_RETURN(pico::cs64_pmr(o, b, op->atb64, op->x64, op->s2, op->cs_lam, op->fista_T, op->theta64.data(), seed,
                                 (uint64_t)(first + done), sigma, atb, y, x, z, tmp, q, acc->sum, acc->sum_im,
                                 acc->sumsq, s));
    done += b;
  }
  acc->count += nrep;
  return PICO_OK;
}

pico_status_t pico_pmr_finalize(pico_op_t op, const pico_accum_t* acc, double* var, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !acc->sum_im || !acc->sumsq || !var)
    return fail(PICO_EINVAL, "NULL accumulator field or output");
  if (acc->count < 2) return fail(PICO_EINVAL, "need at least 2 replicas");
  HIP_OR_RETURN(pico::launch_pmr_finalize(acc->sum, acc->sum_im, acc->sumsq, var,
                                          (int64_t)op->image(), (double)acc->count,
                                          (hipStream_t)stream));
  return PICO_OK;
}

pico_status_t pico_monitor_stderr(pico_op_t op, const pico_accum_t* acc, double* proxy, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !acc->sumsq || !proxy) return fail(PICO_EINVAL, "NULL accumulator field or output");
  if (acc->count < 2) return fail(PICO_EINVAL, "need at least 2 probes");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = (int64_t)op->image();
  const int nblk = (int)std::min<int64_t>(256, (n + 255) / 256);
  std::vector<double> part(2 * nblk);
  HIP_OR_RETURN(pico::launch_stderr_partials(acc->sum, acc->sumsq, (double)acc->count, n, op->mon, nblk, s));
  HIP_OR_RETURN(hipMemcpyAsync(part.data(), op->mon, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OR_RETURN(hipStreamSynchronize(s));
  double num = 0.0, den = 0.0;
  for (int b = 0; b < nblk; ++b) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  *proxy = den > 0.0 ? std::sqrt(num / den) : INFINITY;
  return PICO_OK;
}

pico_status_t pico_noise_map_adaptive(pico_op_t op, uint64_t seed, int64_t first_probe, int64_t max_probes,
                                      double target, int32_t dist, pico_accum_t* acc, pico_stats_t* stats,
                                      int64_t* used, double* proxy, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !acc->sumsq) return fail(PICO_EINVAL, "adaptive stopping needs sum and sumsq buffers");
  if (op->cs) return fail(PICO_EUNSUPPORTED, "adaptive stopping uses the Re(conj v u) terms of CG-SENSE operators");
  if (max_probes < 2 || first_probe < 0) return fail(PICO_EINVAL, "max_probes must be >= 2, first_probe >= 0");
  if (!(target > 0.0)) return fail(PICO_EINVAL, "target must be > 0");
  int64_t done = 0;
  double px = INFINITY;
  pico_stats_t st{}, tot{};
  while (done < max_probes) {
    const int64_t k = std::min<int64_t>(op->K, max_probes - done);
    pico_status_t r = pico_noise_map(op, seed, first_probe + done, k, dist, acc, stats ? &st : nullptr, stream);
    if (r != PICO_OK && r != PICO_ENOTCONV) return r;
    if (stats) {
      tot.max_relres = std::max(tot.max_relres, st.max_relres);
      tot.mean_relres = (tot.mean_relres * (double)tot.probes + st.mean_relres * (double)st.probes) /
                        (double)(tot.probes + st.probes);
      tot.frozen += st.frozen;
      tot.probes += st.probes;
      tot.lambda_abs = st.lambda_abs;
    }
    done += k;
    if (acc->count >= 2) {
      if (pico_status_t e = pico_monitor_stderr(op, acc, &px, stream)) return e;
      if (px <= target) break;
    }
  }
  if (used) *used = done;
  if (proxy) *proxy = px;
  if (stats) {
    *stats = tot;
    if (tot.frozen) return fail(PICO_ENOTCONV, "CG breakdown in " + std::to_string(tot.frozen) + " right-hand side(s)");
  }
  return PICO_OK;
}

pico_status_t pico_monitor_nrmse(pico_op_t op, const pico_accum_t* acc, const double* ref_var,
                                 double* nrmse, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!acc || !acc->sum || !ref_var || !nrmse) return fail(PICO_EINVAL, "NULL accumulator, reference or output");
  if (acc->count < 1) return fail(PICO_EINVAL, "no probes accumulated");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = (int64_t)op->image();
  const int nblk = (int)std::min<int64_t>(256, (n + 255) / 256);
  std::vector<double> part(2 * nblk);
  HIP_OR_RETURN(pico::launch_nrmse_partials(acc->sum, 1.0 / (double)acc->count, ref_var, n,
                                            op->mon, nblk, s));
  HIP_OR_RETURN(hipMemcpyAsync(part.data(), op->mon, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OR_RETURN(hipStreamSynchronize(s));
  double num = 0.0, den = 0.0;
  for (int b = 0; b < nblk; ++b) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  *nrmse = den > 0.0 ? std::sqrt(num / den) : NAN;
  return PICO_OK;
}

pico_status_t pico_init_reduced(const pico_op_desc_t* d, int32_t factor, void* stream, pico_op_t* out) {
  if (!d || !out) return fail(PICO_EINVAL, "NULL descriptor or output handle");
  *out = nullptr;
  if (factor < 2) return fail(PICO_EINVAL, "factor must be >= 2");
  if (d->recon != PICO_CGSENSE)
    return fail(PICO_EUNSUPPORTED, "the reduced grid is built for CG-SENSE operators");
  if (d->ny < 2 || d->nx < 2 || d->ny % factor || d->nx % factor)
    return fail(PICO_EINVAL, "ny and nx must be divisible by the factor");
  const int ny = d->ny, nx = d->nx, nc = d->ncoils, cy = ny / factor, cx = nx / factor;
  if (((ny - cy) & 1) || ((nx - cx) & 1)) return fail(PICO_EINVAL, "the central k-space block must sit on whole samples");
  if (nc < 1 || nc > 64 || !d->maps) return fail(PICO_EINVAL, "maps and ncoils in 1..64 required");
  hipStream_t s = (hipStream_t)stream;
  pico_op_desc_t c = *d;
  c.ny = cy;
  c.nx = cx;
  float2* maps_c = nullptr;
  uint8_t* mask_c = nullptr;
  float* traj_c = nullptr;
  pico::DevAllocator by_maps, by_mask, by_traj;   // temporaries, from the allocator in effect
  auto tmp_alloc = [](auto** p, size_t bytes, pico::DevAllocator* by) {
    void* raw = nullptr;
    const hipError_t e = pico::dev_alloc(&raw, pico::OffsetArena::round_up(bytes), by);
    *p = static_cast<std::remove_reference_t<decltype(**p)>*>(raw);
    return e;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    pico::dev_free(maps_c, by_maps);
    pico::dev_free(mask_c, by_mask);
    pico::dev_free(traj_c, by_traj);
  };
  auto dev_fail = [&](hipError_t e, const char* what) {
    cleanup();
    if (e == hipErrorOutOfMemory) return fail(PICO_ENOMEM, std::string(what) + ": out of device memory");
    return fail(PICO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = tmp_alloc(&maps_c, (size_t)nc * cy * cx * sizeof(float2), &by_maps)) != hipSuccess) return dev_fail(e, "coarse maps");
  if ((e = pico::launch_subsample_maps((const float2*)d->maps, maps_c, nc, ny, nx, factor, s)) != hipSuccess)
    return dev_fail(e, "coarse maps");
  c.maps = maps_c;
  if (d->sampling == PICO_CART_1D || d->sampling == PICO_CART_2D) {
    if (!d->mask) {
      cleanup();
      return fail(PICO_EINVAL, "NULL mask");
    }
    if (d->sampling == PICO_CART_1D) {
      if ((e = tmp_alloc(&mask_c, cy, &by_mask)) != hipSuccess ||
          (e = hipMemcpyAsync(mask_c, d->mask + (ny - cy) / 2, cy, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return dev_fail(e, "coarse mask");
    } else {
      if ((e = tmp_alloc(&mask_c, (size_t)cy * cx, &by_mask)) != hipSuccess ||
          (e = hipMemcpy2DAsync(mask_c, cx, d->mask + (size_t)((ny - cy) / 2) * nx + (nx - cx) / 2, nx, cx, cy,
                                hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return dev_fail(e, "coarse mask");
    }
    c.mask = mask_c;
  } else if (d->sampling == PICO_NONCART) {
    if (!d->traj || d->nsamples < 1) {
      cleanup();
      return fail(PICO_EINVAL, "non-Cartesian sampling needs traj and nsamples >= 1");
    }
    std::vector<float> t((size_t)2 * d->nsamples), kept;
    if ((e = hipMemcpyAsync(t.data(), d->traj, t.size() * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return dev_fail(e, "trajectory");
    const double lim = M_PI / factor;
    for (int64_t m = 0; m < d->nsamples; ++m) {
      const double wy = t[2 * m], wx = t[2 * m + 1];
      if (wy >= -lim && wy < lim && wx >= -lim && wx < lim) {
        kept.push_back((float)(factor * wy));
        kept.push_back((float)(factor * wx));
      }
    }
    if (kept.empty()) {
      cleanup();
      return fail(PICO_EINVAL, "no sample inside the coarse band");
    }
    if ((e = tmp_alloc(&traj_c, kept.size() * sizeof(float), &by_traj)) != hipSuccess ||
        (e = hipMemcpyAsync(traj_c, kept.data(), kept.size() * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return dev_fail(e, "coarse trajectory");
    c.traj = traj_c;
    c.nsamples = (int64_t)kept.size() / 2;
  }
  const pico_status_t st = pico::init_in_arena(&c, stream, nullptr, out);
  cleanup();
  if (st == PICO_OK) (*out)->reduce_f = factor;
  return st;
}

pico_status_t pico_upsample_map(pico_op_t op, const double* coarse, double* var, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (op->reduce_f < 2) return fail(PICO_EUNSUPPORTED, "pico_upsample_map needs an operator from pico_init_reduced");
  if (!coarse || !var) return fail(PICO_EINVAL, "NULL map");
  HIP_OR_RETURN(pico::launch_upsample_bilinear(coarse, var, op->ny, op->nx, op->reduce_f, (hipStream_t)stream));
  return PICO_OK;
}

pico_status_t pico_exact_diag(pico_op_t op, double* var, void* stream) {
  if (pico_status_t st = check_op(op)) return st;
  if (!var) return fail(PICO_EINVAL, "NULL output");
  if (!op->colmajor) return fail(PICO_EUNSUPPORTED, "exact diagonal needs a phase-encode mask");
  hipStream_t s = (hipStream_t)stream;
  for (int y0 = 0; y0 < op->ny; y0 += op->K) {
    const int k = std::min(op->K, op->ny - y0);
    HIP_OR_RETURN(pico::launch_unit_rows(op->r, k, y0, op->ny, op->nx, s));
    HIP_OR_RETURN(apply_sigma(op, k, pico::C1_FIRST_BUF, 0, 0, 0, s));
    HIP_OR_RETURN(pico::launch_extract_rows(op->x, var, k, y0, op->ny, op->nx, s));
  }
  return PICO_OK;
}

pico_status_t pico_profile_start(pico_op_t op) {
  if (pico_status_t st = check_op(op)) return st;
  op->prof_recs.clear();
  op->ev_used = 0;
  op->prof_on = true;
  return PICO_OK;
}

pico_status_t pico_profile_stop(pico_op_t op, double* ms, int64_t* launches) {
  if (pico_status_t st = check_op(op)) return st;
  op->prof_on = false;
  for (int k = 0; k < PICO_PROF_KINDS; ++k) {
    if (ms) ms[k] = 0.0;
    if (launches) launches[k] = 0;
  }
  for (auto& rec : op->prof_recs) {
    HIP_OR_RETURN(hipEventSynchronize(rec.second.second));
    float t = 0.0f;
    HIP_OR_RETURN(hipEventElapsedTime(&t, rec.second.first, rec.second.second));
    if (ms) ms[rec.first] += t;
    if (launches) launches[rec.first] += 1;
  }
  op->prof_recs.clear();
  op->ev_used = 0;
  return PICO_OK;
}

void pico_destroy(pico_op_t op) {
  if (!op) return;
  (void)hipStreamSynchronize(op->last_stream);
  delete op;
}

}  // extern "C"
