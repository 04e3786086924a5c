// Internal interface between the host runtime (pico_abi.hip, serve.hip) and the kernel
// launchers (*.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>

namespace pico {

// Device allocator in effect for library workspaces: the caller's callbacks
// (pico_set_allocator) or, with both NULL, hipMalloc / hipFree.  Each
// allocation remembers the allocator that made it, so it is returned to the
// same one even if the caller installs another in between.
struct DevAllocator {
  void* (*alloc)(size_t bytes, void* ctx) = nullptr;
  void (*free)(void* ptr, void* ctx) = nullptr;
  void* ctx = nullptr;
};
// Allocates `bytes` (256-byte aligned) with the allocator in effect, which it
// reports in *by; hipErrorOutOfMemory when the callback returns NULL, and
// hipErrorInvalidValue for a pointer that is not 256-byte aligned (it is
// handed back to the callback first).
hipError_t dev_alloc(void** ptr, size_t bytes, DevAllocator* by);
void dev_free(void* ptr, const DevAllocator& by);

// Per-probe CG state flags
enum : int { CG_ACTIVE = 0, CG_CONVERGED = 1, CG_BREAKDOWN = 2 };

// Modes of the separable Cartesian column kernel.
enum Cart1dMode : int {
  C1_FIRST_PROBE = 0,  // r = p = v (Philox probe); q = (M + lam) p
  C1_FIRST_BUF = 1,    // p = r (right-hand side already in r); q = (M + lam) p
  C1_ITER = 2,         // x += alpha p, r -= alpha q, p = r + beta p; q = (M + lam) p
  C1_APPLY = 3,        // dst = (M + lam) (scale * src)
  C1_PMR_RHS = 4,      // r = A^H n, n white k-space noise in the hybrid (ky, x) domain
};

struct Cart1dArgs {
  int ny, nx, nc, K;           // K probes in this launch
  const float2* maps;          // [nx][nc][ny] whitened, (-1)^y folded
  const uint32_t* maps_bf;     // the same maps as packed bfloat16 pairs, or NULL
  const float* maskw;          // [ny] weight mask[k] / ny (0 off the mask)
  const float2* twt;           // [ny] W_ny^m = exp(-2 pi i m / ny)
  const float2* src;           // input field   (mode dependent)
  float2* x;                   // [K][nx][ny]
  float2* r;
  float2* p;
  float2* q;
  const double* alpha;         // [K] step of the previous iteration
  const double* beta;          // [K]
  int x_zero;                  // C1_ITER: x enters as 0 (first update)
  double* part;                // [K][nx][4]: |r|^2, Re p^H q, |q|^2, Re r^H q
  float lam;                   // added to M p
  float scale;                 // C1_APPLY input scale
  uint64_t seed, first;        // probe / noise draw
  const uint64_t* tp;          // non-NULL: (seed, first) read from device memory here
  int dist;                    // probe family
};

// Last CG update x += alpha p
struct FinalArgs {
  int n, K;                    // n = voxels per probe
  float2* x;
  const float2* p;
  const double* alpha;         // [K]
  int x_zero;                  // x enters as 0 (single-iteration solves)
};

struct ScalarArgs {
  int K, nblk;
  const double* part;          // [K][nblk][4]: |r_i|^2, Re p_i^H q_i, |q_i|^2, Re r_i^H q_i
  double* alpha;               // [K]
  double* beta;                // [K]
  double* rr;                  // [K] |r_{i+1}|^2
  double* rr0;                 // [K]
  int* state;                  // [K]
  double tol;
  int first;                   // 1 after the first normal-operator application
};

struct AccumArgs {
  int ny, nx, K;
  const float2* x;             // [K][nx][ny] (col-major image per probe)
  double* sum;                 // [ny*nx]
  double* sum_im;              // may be null
  double* sumsq;               // may be null
  uint64_t seed, first;
  const uint64_t* tp;          // non-NULL: (seed, first) read from device memory here
  int dist;
  int pmr;                     // 1: accumulate x itself (PMR); 0: conj(v) x (PICO)
};

// 2-D grid normal operator (Cartesian 2-D masks, Toeplitz non-Cartesian)
struct Grid2dArgs {
  int ny, nx, nc, K, Gy, Gx;
  const float2* maps;          // [nc][ny][nx] whitened (and sign-folded for Cartesian)
  const uint32_t* maps_bf;     // the same maps as packed bfloat16 pairs, or NULL
  const float* w;              // [Gx][Gy] real weights
  const float2* twx;           // [Gx] W_Gx^m
  const float2* twy;           // [Gy] W_Gy^m
  float2* T;                   // [K][nc][ny][Gx] row-transformed planes
  uint32_t* Tb;                // non-NULL: T kept as packed bfloat16 pairs here instead
  const float2* src;           // C1_APPLY input [K][ny][nx]
  float2* x;                   // [K][ny][nx]
  float2* r;
  float2* p;
  float2* q;
  const double* alpha;
  const double* beta;
  int x_zero;
  double* part;                // [K][ny][4]
  float lam, scale;
  uint64_t seed, first;
  const uint64_t* tp;          // non-NULL: (seed, first) read from device memory here
  int dist;
};

bool cart1d_supported(int ny);
bool grid_line_supported(int n);
size_t grid_cols_lds_bytes(int Gy, int ny);
hipError_t launch_grid_normal(int mode, const Grid2dArgs& a, hipStream_t s);
hipError_t launch_grid_normal_bf16(int mode, const Grid2dArgs& a, hipStream_t s);   // a.maps_bf set
hipError_t launch_accum_rowmajor(const AccumArgs& a, hipStream_t s);
hipError_t launch_prep_maps_rowmajor(const float2* maps, const double* linv, float2* out, int nc,
                                     int ny, int nx, int fold, hipStream_t s);
hipError_t launch_mask_weights(const uint8_t* mask, float* w, int ny, int nx, float scale,
                               hipStream_t s);
// bf = maps rounded to bfloat16 (nearest even); round_copy: maps too become
// the rounded values (the FP32 copy then describes the same operator)
hipError_t launch_quantise_maps(float2* maps, uint32_t* bf, long count, bool round_copy, hipStream_t s);
// reduced-resolution grid: maps [nc][ny][nx] -> [nc][ny/f][nx/f] at native pixels
// (f my, f mx); coarse map [cy][cx] -> [f cy][f cx] by periodic bilinear weights
hipError_t launch_subsample_maps(const float2* maps, float2* out, int nc, int ny, int nx, int f, hipStream_t s);
hipError_t launch_upsample_bilinear(const double* coarse, double* out, int cy, int cx, int f, hipStream_t s);
hipError_t launch_power_start_rowmajor(float2* p, int n, hipStream_t s);
hipError_t launch_fft2d(float2* data, long planes, int ny, int nx, bool inverse, const float2* twx,
                        const float2* twy, hipStream_t s);
// gridding normal operator passes on the ny image rows of a Gy x Gx grid
// (image row y at grid row (y - ny/2) mod Gy, column x at (x - nx/2) mod Gx):
// forward rows: out [K][ny][Gx] = row FFTs of S_c x dy dx scale placed on the
// grid rows; inverse rows: out [K][ny][nx] (= or +=, accumulate) conj(S_c)
// dy dx scale times the inverse row FFTs of in [K][ny][Gx], cropped.
// Column transforms: forward [planes][ny][Gx] (the image rows) -> the full
// [planes][Gy][Gx]; inverse the full grid -> its image rows [planes][ny][Gx].
hipError_t launch_kbn_rows(bool inverse, const float2* in, const float2* Sc, const float* dy, const float* dx,
                           float2* out, int K, int ny, int nx, int Gx, float scale, int accumulate,
                           const float2* twx, hipStream_t s);
hipError_t launch_fft_cols_crop(const float2* in, float2* out, long planes, int ny, int Gy, int Gx, bool inverse,
                                const float2* twy, hipStream_t s);
hipError_t launch_kspace_in(const float2* src, const double* linv, const uint8_t* mask, float2* out,
                            int B, int nc, int ny, int nx, uint64_t seed, uint64_t first,
                            const uint64_t* tp, uint32_t stream, int dist, float scale, hipStream_t s);
hipError_t launch_coil_combine(const float2* T, const float2* maps, float2* out, int B, int nc,
                               long n, hipStream_t s);
// CS tangents: analysis of the gradient point y - (q - g) * inv_s2 into dst
// with the soft-threshold derivative at ck on the details (scratch holds the
// coarser levels' inputs); synthesis of src (read only; scratch for the
// coarser levels) with the FISTA momentum into (xo, y)
hipError_t launch_cs_analysis(const float2* y, const float2* q, const float2* g, float inv_s2, float2* scratch,
                              float2* dst, int K, int ny, int nx, int levels, const double2* ck, double lam,
                              hipStream_t s);
hipError_t launch_cs_synthesis(const float2* src, float2* scratch, int K, int ny, int nx, int levels, float2* xo,
                               float2* y, float theta, hipStream_t s);
hipError_t launch_fista_grad(const float2* y, const float2* q, const float2* g, float2* z, long n, int K,
                             int gK, float inv_s2, hipStream_t s);
hipError_t launch_momentum(const float2* xn, float2* xo, float2* y, long total, float theta,
                           hipStream_t s);
hipError_t launch_accum_abs2(const float2* u, double* sum, double* sum_im, double* sumsq, int K, long n,
                             hipStream_t s);
hipError_t launch_fill_zero(float2* a, long total, hipStream_t s);
size_t toeplitz_scratch_bytes(long M, int ny, int nx);
// synchronous on s; scratch: toeplitz_scratch_bytes(M, ny, nx) bytes of device memory
hipError_t build_toeplitz_weights(const float* traj, long M, int ny, int nx, float* w, void* scratch,
                                  hipStream_t s);
// complex128 GEMM (row-major; flags 1 transA, 2 conjA, 4 conjB; split-K slices
// land in C[slice]); batch b offsets A, B, C by b * sA, sB, sC
hipError_t zgemm64(const double2* A, const double2* B, double2* C, int Mr, int Nc, int Kd,
                   int flags, int splits, hipStream_t s, int batch = 1, long sA = 0, long sB = 0,
                   long sC = 0);

// FP64 compressed-sensing primal (2-D Cartesian): the normal operator by dense
// centred-DFT products, power method, FISTA storing its wavelet coefficients
constexpr int CS64_DOT_BLOCKS = 1024;
struct Cs64 {
  int ny = 0, nx = 0, nc = 0, levels = 0;
  double2* S = nullptr;         // [nc][ny][nx] whitened coil maps
  double2* Fy = nullptr;        // [ny][ny] centred orthonormal DFT
  double2* Fx = nullptr;        // [nx][nx]
  const uint8_t* mask = nullptr;  // [ny][nx]
  double2* U = nullptr;         // [B][nc][ny][nx] workspace (B images per call)
  double2* V = nullptr;         // [B][nc][ny][nx] workspace
  // proximal step: the L1 wavelet threshold (tv_inner = 0) or TV by tv_inner
  // dual fast-gradient-projection steps with momentum weights tv_th (host)
  int tv_inner = 0;
  const double* tv_th = nullptr;
  double2* tv_r = nullptr;      // [B][2][ny][nx] dual workspace
  double2* tv_p = nullptr;      // [B][2][ny][nx]
  double2* tv_u = nullptr;      // [B][ny][nx]
  // primal trajectory stored for the tangents (B = 1 with store): wavelet
  // c_k = Psi z_k [T][ny][nx], or the TV projection data [T][tv_inner][ny][nx]
  double2* ctraj = nullptr;
  float4* tv_what = nullptr;
  float* tv_invn = nullptr;
};
hipError_t cs64_setup(Cs64& o, const float2* maps, const double* linv, hipStream_t s);
hipError_t cs64_normal(const Cs64& o, int B, const double2* y, double2* q, hipStream_t s);
hipError_t cs64_adjoint_kdata(const Cs64& o, const float2* kdata, const double* linv, double2* out,
                              hipStream_t s);
hipError_t cs64_power(const Cs64& o, int iters, double2* v, double2* w, double* part_d, double* out,
                      hipStream_t s);
hipError_t cs64_fista(const Cs64& o, int B, const double2* atb, double s2, double lam, int T,
                      const double* theta, bool store, double2* y, double2* x, double2* z,
                      double2* tmp, double2* q, hipStream_t s);
hipError_t cs64_pmr(const Cs64& o, int B, const double2* atb0, const double2* x0, double s2, double lam,
                    int T, const double* theta, uint64_t seed, uint64_t first, double sigma, double2* atb,
                    double2* y, double2* x, double2* z, double2* tmp, double2* q, double* sum,
                    double* sum_im, double* sumsq, hipStream_t s);
hipError_t launch_to_f32(const double2* a, float2* b, long n, hipStream_t s);
// TV prox of B FP64 images in place (o.tv_* workspace); what / invn: the
// projection data of its o.tv_inner steps ([tv_inner][ny][nx]) or NULL
hipError_t tv64_prox(const Cs64& o, int B, double2* z, double lam, float4* what, float* invn, hipStream_t s);
// tangent of one TV FISTA step for K FP32 images: the prox's inner steps on
// dz (kept), fused several per pass, with the ping-pong pairs drA / drB and
// dpA / dpB ([K][2][n] each), the last pass also forming the prox output
// dx = dz - lam D^H dp and the FISTA momentum yo = dx + theta (dx - xo),
// xo = dx.  Needs ny >= 13 and nx >= 37; passes of four steps need ny >= 25
// and nx >= 41 (smaller images take pairs only).
hipError_t tv_tangent_step(const float2* dz, float2* drA, float2* drB, float2* dpA, float2* dpB,
                           const float4* what, const float* invn, int ny, int nx, int K, int inner,
                           const float* th, float lam, float2* xo, float2* yo, float theta, hipStream_t s);

// Kaiser-Bessel gridding NUFFT (non-Cartesian data path)
// Kaiser-Bessel gridding tables: samples sorted into square bins of
// kKbTile x kKbTile grid cells by the cell of their first tap, so that every
// grid tile finds the samples whose footprint reaches it in its own bin and
// the three bins below / left of it.
constexpr int kKbTile = 8;
// The gridding normal operator applies P^H P (P the interpolation from the
// grid to the samples) as a precomputed real stencil over (2W - 1)^2 grid
// offsets, stored for the kKbStencilTile^2-point tiles that any sample's
// footprint reaches ("active" tiles); the others stay zero.
constexpr int kKbStencilTile = 16;
struct KbLayout {
  static constexpr int kParts = 13;   // sky0 skx0 swy swx perm bin_ptr dy dx twx twy grid grid2 stencil+list
  size_t sizes[kParts];
  size_t bytes_of(size_t i) const;
};
// normal: also the second grid and the stencil of the gridding normal
// operator (room for every tile: which ones are active depends on the
// trajectory, and the byte count must follow from the description alone)
KbLayout kb_layout(long M, int W, int ny, int nx, int Gy, int Gx, int K, bool normal);
struct KbOp {
  long M = 0;
  int W = 0, ny = 0, nx = 0, Gy = 0, Gx = 0;
  int nby = 0, nbx = 0;                 // bins per axis (G / kKbTile)
  int *sky0 = nullptr, *skx0 = nullptr; // [M] first tap cell per axis (mod G), bin order
  float *swy = nullptr, *swx = nullptr; // [M][W] tap weights, bin order
  int* perm = nullptr;                  // [M] sample index of each position in bin order
  int* bin_ptr = nullptr;               // [nby nbx + 1] first position of each bin
  float *dy = nullptr, *dx = nullptr;   // de-apodisation [ny], [nx]
  float2 *twx = nullptr, *twy = nullptr;
  float2* grid = nullptr;               // [K][Gy][Gx]
  float2* grid2 = nullptr;              // [K][Gy][Gx], gridding normal operator only
  // gridding normal operator: stencil tiles, active ones first
  int n_active = 0;
  int* tile_list = nullptr;             // [(Gy / 16) (Gx / 16)] tile of each slot
  float* stencil = nullptr;             // [n_active][(2W - 1)^2][256] P^H P per offset and point
                                        // (room for every tile)
};
double kb_beta(double sigma, int W);
// host tables in bin order (double precision, stored float32); traj_h [M][2]
void kb_build_host(const float* traj_h, long M, int W, double sigma, int ny, int nx, int Gy, int Gx,
                   std::vector<int>& sky0, std::vector<int>& skx0, std::vector<float>& swy,
                   std::vector<float>& swx, std::vector<int>& perm, std::vector<int>& bin_ptr,
                   std::vector<float>& dy, std::vector<float>& dx);
// stencil of P^H P in FP64 from the tap tables above (bin order), stored FP32
// [n_active][(2W - 1)^2][256]; tile_list: active tiles first, in tile order
void kb_build_stencil(const std::vector<int>& sky0, const std::vector<int>& skx0, const std::vector<float>& swy,
                      const std::vector<float>& swx, long M, int W, int Gy, int Gx, std::vector<int>& tile_list,
                      int& n_active, std::vector<float>& stencil);
hipError_t kb_adjoint(const KbOp& o, const float2* maps, int nc, int K, const float2* src, uint64_t seed,
                      uint64_t first, float2* out, hipStream_t s);
hipError_t kb_forward(const KbOp& o, const float2* maps, int nc, int K, const float2* x, float2* out,
                      hipStream_t s);
// Gridding normal operator q = (sum_c S_c^H A_c^H A_c S_c + lam) p with the
// Kaiser-Bessel A_c (interpolation and spread fused per grid tile), in the
// CG modes and with the partial dots of launch_grid_normal
hipError_t launch_kb_normal(int mode, const Grid2dArgs& a, const KbOp& o, hipStream_t s);
hipError_t launch_cart1d(int mode, const Cart1dArgs& a, hipStream_t s);
hipError_t launch_cart1d_bf16(int mode, const Cart1dArgs& a, hipStream_t s);   // a.maps_bf set
// dense per-column normal operator (phase-encode masks, FP32 matrix cores)
bool gram_supported(int ny);
size_t gram_bytes(int ny, int nx);
hipError_t build_gram(const float2* maps, const float* maskw_h, int nc, int ny, int nx, float2* G,
                      double2* cvec_d, hipStream_t s);
hipError_t launch_cart1d_gram(int mode, const Cart1dArgs& a, const float2* G, hipStream_t s);
// the same blocks split into FP16 pairs for the FP16 matrix cores: G16 has
// gram_bytes / 4 words, gexp nx column exponents, pexp gram16_pexp_count ints
size_t gram16_pexp_count(int nx, int K);
hipError_t build_gram16(const float2* maps, const float* maskw_h, int nc, int ny, int nx, uint32_t* G16, int* gexp,
                        double2* cvec_d, hipStream_t s);
hipError_t launch_cart1d_gram16(int mode, const Cart1dArgs& a, const uint32_t* G16, const int* gexp, int* pexp,
                                hipStream_t s);
// device (seed, first) of the next replayed probe tile
hipError_t launch_set_tile(uint64_t* tp, uint64_t seed, uint64_t first, hipStream_t s);
hipError_t launch_final_x(const FinalArgs& a, hipStream_t s);
hipError_t launch_scalars(const ScalarArgs& a, hipStream_t s);
hipError_t launch_accum_colmajor(const AccumArgs& a, hipStream_t s);
hipError_t launch_prep_maps_cart1d(const float2* maps, const double* linv, float2* out,
                                   int nc, int ny, int nx, hipStream_t s);
hipError_t launch_transpose_in(const float2* v, float2* out, int K, int ny, int nx, hipStream_t s);
hipError_t launch_transpose_out(const float2* x, float2* u, int K, int ny, int nx, hipStream_t s);
hipError_t launch_finalize(const double* sum, double* var, int64_t n, double inv_count,
                           hipStream_t s);
hipError_t launch_pmr_finalize(const double* sum, const double* sum_im, const double* sumsq,
                               double* var, int64_t n, double count, hipStream_t s);
hipError_t launch_power_start(float2* p, int ny, int nx, hipStream_t s);
hipError_t launch_unit_rows(float2* r, int K, int y0, int ny, int nx, hipStream_t s);
hipError_t launch_extract_rows(const float2* x, double* var, int K, int y0, int ny, int nx,
                               hipStream_t s);
hipError_t launch_stderr_partials(const double* sum, const double* sumsq, double count, int64_t n,
                                  double* part, int nblk, hipStream_t s);
hipError_t launch_nrmse_partials(const double* sum, double inv_count, const double* ref, int64_t n,
                                 double* part, int nblk, hipStream_t s);

}  // namespace pico
