/*
 * pico.h - C ABI of libpico: voxelwise noise-variance maps of iterative MRI
 * reconstructions by image-space covariance probing (PICO), on AMD Instinct
 * MI355X (gfx950).
 *
 * Method (Dalmaz et al., "Fast Voxelwise SNR Estimation for Iterative MRI
 * Reconstructions"):
 *   - pre-whitened encoding A = L^-1 A~ with L L^H = Sigma_n (Sec. 2.1, Eq. (3));
 *   - CG-SENSE reconstruction x = (A^H A + lam I)^-1 A^H b_w (Sec. 2.1, Eqs. (5)-(6));
 *   - image covariance Sigma = (M + lam)^-1 M (M + lam)^-1, M = A^H A
 *     (Sec. 2.1, Eqs. (7)-(9)), applied implicitly with CG solves
 *     (Sec. 2.2, "Implicit matrix-vector product via CG");
 *   - diagonal estimate var = Re((1/N) sum_i conj(v_i) . Sigma v_i) over
 *     random-phase probes v_i (Sec. 2.2, Eqs. (13)-(14), (20); App. A,
 *     Algorithm 1);
 *   - the pseudo-multiple-replica baseline (Sec. 1; App. C).
 *
 * Conventions shared by every entry point:
 *   - complex data are interleaved float32 pairs (complex64); images are
 *     row-major [ny][nx]; multi-coil arrays are [ncoils][ny][nx];
 *   - k-space masks are given in centred order (DC at index n/2), and the
 *     Fourier transform is the centred orthonormal DFT;
 *   - "device" pointers are HIP device memory (e.g. torch.Tensor.data_ptr()
 *     of a CUDA/ROCm tensor); "host" pointers are ordinary memory;
 *   - ``stream`` is a hipStream_t passed as void* (NULL = default stream);
 *     every call enqueues its work on that stream and returns without
 *     waiting, except pico_init (synchronous) and calls given a non-NULL
 *     stats pointer (which wait for the stream);
 *   - the library never frees caller memory; caller buffers must stay alive
 *     until the enqueued work has finished;
 *   - every function returns a status; on anything but PICO_OK,
 *     pico_last_error() returns a message (thread-local).  Argument errors
 *     are detected before anything is enqueued.
 *   - one host thread per pico_op_t at a time; distinct handles are
 *     independent.
 */
#ifndef PICO_H_
#define PICO_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pico_op_s* pico_op_t;

typedef enum {
  PICO_OK = 0,
  PICO_EINVAL = 1,         /* invalid argument or unsupported shape            */
  PICO_ENOMEM = 2,         /* device allocation failed (nothing leaked)        */
  PICO_EDEVICE = 3,        /* HIP runtime error                                */
  PICO_EUNSUPPORTED = 4,   /* valid request this build does not implement      */
  PICO_ENOTCONV = 5        /* some CG right-hand side broke down (map written) */
} pico_status_t;

typedef enum {
  PICO_CART_1D = 0,        /* Cartesian, phase-encode mask [ny], all kx sampled */
  PICO_CART_2D = 1,        /* Cartesian, 2-D mask [ny][nx]                     */
  PICO_NONCART = 2         /* non-Cartesian trajectory                         */
} pico_sampling_t;

typedef enum {
  PICO_CGSENSE = 0,        /* linear Tikhonov / least-squares CG-SENSE          */
  PICO_CS_FISTA_L1WAV = 1, /* nonlinear compressed sensing, L1 on db4 wavelet
                              details (Jacobian probing)                        */
  PICO_CS_FISTA_TV = 2     /* nonlinear compressed sensing, isotropic total
                              variation (Sec. 3.2.3 model; Jacobian probing)    */
} pico_recon_t;

typedef enum {
  PICO_RANDOM_PHASE = 0,   /* v = exp(j 2 pi f), Sec. 2.2 Eq. (20) (default)    */
  PICO_QPSK = 1,           /* v in {1, j, -1, -j}                               */
  PICO_RADEMACHER = 2,     /* v in {+1, -1}, Sec. 2.2 Eq. (19)                  */
  PICO_GAUSSIAN = 3        /* v ~ CN(0, 1), Sec. 2.2 Eq. (18)                   */
} pico_probe_t;

typedef enum {
  PICO_FP32 = 0,           /* complex64 maps and intermediates (default)        */
  PICO_BF16_MAPS = 1,      /* whitened maps rounded to bfloat16 (nearest even)
                              and stored packed.  CG-SENSE: the operator is the
                              one of the rounded maps on every path.  Compressed
                              sensing: only the tangents' normal-operator reads
                              use them; the FP64 reconstruction (the point the
                              Jacobian is taken at) and the probes' k-space
                              adjoint keep the unrounded maps                     */
  PICO_BF16_STREAM = 2     /* as 1, plus the row-transformed coil planes of the
                              2-D grid path (Cartesian 2-D, Toeplitz) stored as
                              bfloat16 between its passes; arithmetic, CG vectors,
                              dots and accumulators stay FP32 / FP64            */
} pico_storage_t;

/* Operator description.  Pointers are read during pico_init only. */
typedef struct {
  int32_t ny, nx, ncoils;       /* image size and coil count (1..64)              */
  const void* maps;             /* device complex64 [ncoils][ny][nx], un-whitened */
  const double* psi;            /* host complex128 [ncoils][ncoils] (re, im
                                   interleaved), channel noise covariance Sigma_n
                                   (Sec. 2.1, Eq. (2)); NULL = identity            */
  int32_t sampling;             /* pico_sampling_t                                 */
  const uint8_t* mask;          /* device uint8, [ny] for PICO_CART_1D or [ny][nx]
                                   for PICO_CART_2D, centred order, 0 / 1          */
  const float* traj;            /* device float32 [nsamples][2] (w_y, w_x) rad in
                                   [-pi, pi), PICO_NONCART only                    */
  int64_t nsamples;
  double lambda;                /* Tikhonov weight relative to the normalised
                                   operator (Sec. 3.2.2); >= 0                     */
  int32_t cg_iters;             /* CG iterations per solve (>= 1)                  */
  double cg_tol;                /* 0: exactly cg_iters; > 0: stop a right-hand side
                                   once ||r|| / ||r0|| <= cg_tol                   */
  int32_t power_iters;          /* power-method steps for lambda_max (paper: 15)   */
  double power_margin;          /* safety factor on lambda_max (paper: 1.01)       */
  int32_t probe_tile;           /* probes solved together (K); sizes the workspace */
  int32_t recon;                /* pico_recon_t                                    */
  /* PICO_CS_FISTA_L1WAV and PICO_CS_FISTA_TV (Sec. 2.2 CS extension,
   * Sec. 3.2.3): */
  const void* kdata;            /* device complex64 [ncoils][ny][nx] measured
                                   k-space (un-whitened, centred order)            */
  int32_t fista_iters;          /* FISTA iterations T (paper: 100)                 */
  double cs_lambda;             /* L1 / TV weight of the normalised problem
                                   (paper's TV weight: 1e-2)                        */
  int32_t wavelet_levels;       /* L1WAV: db4 levels; ny, nx divisible by 2^levels */
  /* PICO_NONCART data path (A, A^H of sample arrays; PMR replicas) by a
   * Kaiser-Bessel gridding NUFFT (Sec. 3.2.2, 3.3); kb_width = 0 builds none.
   * Grid oversamp * n per axis (an integer with a built FFT length), kernel
   * I0(beta sqrt(1 - (2u/W)^2)), beta = pi sqrt((W/oversamp)^2 (oversamp -
   * 1/2)^2 - 0.8), W = kb_width even in 2..8.  The normal operator of the
   * CG solves is the exact Toeplitz form unless noncart_normal = 1. */
  double oversamp;              /* e.g. 2.0 (or 1.25)                             */
  int32_t kb_width;             /* e.g. 6 (or 4); 0 = no gridding data path       */
  /* Form of the normal operator for PICO_CART_1D (M is block diagonal over
   * image columns, Sec. 2.1 Eq. (6)): 1 = column FFTs; 2 = the dense ny x ny
   * block of every column, built once (nx ny^2 complex64 of device memory)
   * and applied to the probe tile on the FP32 matrix cores (ny a multiple
   * of 32, <= 512); 3 = the same blocks applied on the FP16 matrix cores
   * with each FP32 operand split into two FP16 parts and three partial
   * products accumulated in FP32 (Ootomo and Yokota 2022), operands scaled
   * by powers of two per column block and per probe (the same device
   * memory as 2, plus nx * ceil(probe_tile / 32) * 32 ints of exponents);
   * 0 = the default (column FFTs).
   * Forms 1 and 2 give M to FP32 rounding, form 3 to about 2.4 times that
   * (the split keeps 22 significand bits of each operand); the PMR
   * right-hand side always uses FFTs. */
  int32_t normal_form;
  /* PICO_CS_FISTA_TV: dual fast-gradient-projection steps per proximal step
   * (Beck and Teboulle 2009), from a zero dual start each FISTA iteration,
   * 1..1000.  The tangents keep the projection data of every step of the
   * primal: fista_iters * tv_inner_iters * ny * nx * 20 bytes of device
   * memory.  Needs ny >= 14 and nx >= 38. */
  int32_t tv_inner_iters;
  /* pico_storage_t: precision of stored maps and streamed intermediates
   * (mixed precision; bfloat16 results agree with FP32 storage to about
   * 1e-2 relative). */
  int32_t storage;
  /* 1: pico_noise_map runs each probe tile as one HIP graph (the tile's whole
   * kernel sequence: probe draw, every CG iteration, the Tikhonov middle
   * product or the CS tangent iterations, the FP64 accumulation), captured on
   * first use per (tile size, probe family, accumulator buffers) and
   * replayed with the tile's (seed, first probe) read from device memory;
   * results are bitwise those of direct launches.  Up to 8 graphs per
   * operator are kept (least recently used evicted).  Not used while kernel
   * profiling is on (pico_profile_start).  0: direct launches. */
  int32_t graph;
  /* PICO_NONCART: normal operator of the CG solves.  0: the exact Toeplitz
   * form (point-spread function by the direct NUDFT).  1: the gridding form
   * M = sum_c S_c^H A_c^H A_c S_c with the Kaiser-Bessel A_c of oversamp /
   * kb_width (kb_width > 0, oversamp * n a multiple of 16): per coil and
   * probe, the image rows expanded and row-transformed, column transforms to
   * the full grid, interpolation followed by spread applied as one real
   * stencil per 16 x 16 grid tile (P^H P, built once from the binned
   * samples), and the inverse transforms back to the image rows, cropped
   * and combined; deterministic. */
  int32_t noncart_normal;
} pico_op_desc_t;

/* Caller-owned device float64 accumulators, each [ny*nx] row-major, and a
 * host probe count that the library advances.  Zero them before the first
 * call.  sum_im and sumsq may be NULL.  For a CS operator pico_noise_map
 * accumulates sum |u|^2, sum Re u and sum |u|^4 with u = J w (k-space
 * random-phase probes, Philox stream 2, element (c ny + ky) nx + kx). */
typedef struct {
  double* sum;                  /* PICO: sum Re(conj v . u); PMR: sum Re x         */
  double* sum_im;               /* PICO: sum Im(conj v . u); PMR: sum Im x         */
  double* sumsq;                /* PICO: sum (Re(conj v . u))^2; PMR: sum |x|^2    */
  int64_t count;                /* probes / replicas accumulated                   */
} pico_accum_t;

typedef struct {
  int64_t probes;               /* right-hand sides solved by the call             */
  double max_relres;            /* max over them of ||r|| / ||r0|| at exit         */
  double mean_relres;
  int32_t frozen;               /* right-hand sides stopped by a CG breakdown       */
  double lambda_abs;            /* lambda * power_margin * lambda_max              */
} pico_stats_t;

/* Device allocator for every library workspace, so that the caller (e.g.
 * PyTorch's caching allocator) owns all device memory.  alloc(bytes, ctx) returns device memory of the current device, aligned to
 * 256 bytes, or NULL on failure (the calling entry point then reports
 * PICO_ENOMEM, or PICO_EDEVICE for a misaligned pointer, which is handed back
 * to free first); free_fn(ptr, ctx) releases it.  Every later allocation of
 * pico_init, pico_init_reduced (its temporaries included), pico_pmr_cs (its
 * replica workspace) and pico_server_create (the budget) goes through them,
 * and each block returns to the pair (and ctx) that made it, even if another
 * pair is installed meanwhile.  The library frees a block only after the work
 * it enqueued on it has finished (pico_destroy waits for the operator's last
 * stream).  Both NULL restores hipMalloc / hipFree (the default).  The
 * callbacks may run on any thread that calls into the library and must not
 * call back into it.  Process-wide; takes effect for allocations made after
 * it returns.  Errors: PICO_EINVAL when exactly one callback is NULL. */
pico_status_t pico_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_fn)(void* ptr, void* ctx),
                                 void* ctx);

/* Build the operator: whitens the maps (Cholesky of psi on the host in
 * float64; Sec. 2.1 Eq. (3)), prepares the sampling structures, runs the
 * power method when lambda > 0 (Sec. 3.2.1, 3.3) and allocates the CG
 * workspace for probe_tile right-hand sides.  Synchronous on ``stream``.
 * Errors: PICO_EINVAL for a NULL or malformed descriptor (ny, nx even and
 * supported by a built FFT size, 1 <= ncoils <= 64, cg_iters >= 1,
 * probe_tile >= 1, psi Hermitian positive definite), PICO_EUNSUPPORTED for a
 * sampling / reconstruction kind not built, PICO_ENOMEM, PICO_EDEVICE. */
pico_status_t pico_init(const pico_op_desc_t* desc, void* stream, pico_op_t* out);

/* u = Sigma v for k probe images (Sec. 2.2, Eq. (12)): v, u device
 * complex64 [k][ny][nx], 1 <= k <= probe_tile, v and u may not overlap.
 * Errors: PICO_EINVAL (NULL, k out of range), PICO_ENOTCONV (a right-hand
 * side broke down; u still written), PICO_EDEVICE. */
pico_status_t pico_apply_cov(pico_op_t op, const void* v, void* u, int32_t k, void* stream);

/* u = J w for k whitened k-space probes w (device complex64 [k][ncoils][ny][nx],
 * centred order; entries off the mask are ignored), J the Jacobian of the
 * T-iteration FISTA reconstruction at the operator's data (Sec. 2.2, CS
 * extension); u device complex64 [k][ny][nx].  Errors: PICO_EUNSUPPORTED on a
 * CG-SENSE operator (use pico_apply_cov), PICO_EINVAL (NULL, k out of range). */
pico_status_t pico_apply_jvp(pico_op_t op, const void* w, void* u, int32_t k, void* stream);

/* The reconstruction itself, x (device complex64 [ny][nx]): the FISTA result
 * at the operator's data for a CS operator.  PICO_EUNSUPPORTED otherwise. */
pico_status_t pico_recon(pico_op_t op, void* x, void* stream);

/* Add probes [first_probe, first_probe + nprobes) of the counter-based
 * probe sequence ``seed`` into ``acc`` (App. A, Algorithm 1).  Probe i,
 * voxel j (row-major) is Philox4x32-10(counter = (j, i mod 2^32, i >> 32, 0),
 * key = (seed mod 2^32, seed >> 32)) mapped to the family ``dist``; random
 * phase uses f = (word0 >> 8) / 2^24, v = exp(j 2 pi f).  Splitting a probe
 * range across calls gives the same map (bitwise when the split points are
 * multiples of probe_tile).  stats may be NULL (no wait).
 * Errors: PICO_EINVAL (NULL op / acc / acc->sum, nprobes < 0, bad dist),
 * PICO_ENOTCONV, PICO_EDEVICE. */
pico_status_t pico_noise_map(pico_op_t op, uint64_t seed, int64_t first_probe, int64_t nprobes,
                             int32_t dist, pico_accum_t* acc, pico_stats_t* stats, void* stream);

/* var = sum / count (device float64 [ny*nx]); Algorithm 1, last step.
 * Errors: PICO_EINVAL (count < 1). */
pico_status_t pico_finalize(pico_op_t op, const pico_accum_t* acc, double* var, void* stream);

/* Pseudo multiple replica baseline: replicas [first, first + nrep) of white
 * k-space noise n ~ CN(0, I) (Philox stream 1, Box-Muller), reconstructed by
 * the same CG-SENSE solve, accumulated as sum x (sum / sum_im) and sum |x|^2
 * (sumsq, required).  For a phase-encode (1-D) mask the noise is drawn in the
 * hybrid (ky, x) domain, which the unitary DFT along x leaves white.
 * Errors: as pico_noise_map; sum_im and sumsq must be non-NULL. */
pico_status_t pico_pmr_baseline(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep,
                                pico_accum_t* acc, pico_stats_t* stats, void* stream);

/* pico_pmr_cs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same replicas, batches and sums as pico_pmr_cs (bitwise), with the
 * replica workspace in a fixed 64 MiB device array of the library (one per
 * GPU, held until the process ends) instead of device memory allocated on
 * the first call.  The workspace of B = min(probe_tile, 16) replicas,
 * B (2 ncoils + 6) ny nx 16 bytes (TV: B (2 ncoils + 11) ny nx 16), must fit
 * in it: larger operators get PICO_EINVAL and nothing is enqueued.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (any operator, any stream) race: a caller must
 * order them (one stream, or events).  Errors: as pico_pmr_cs. */
pico_status_t pico_pmr_cs_noalloc(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep, double sigma,
                                  pico_accum_t* acc, void* stream);

/* Unbiased replica variance (sumsq - |sum|^2 / N) / (N - 1) into var
 * (device float64 [ny*nx]).  Errors: PICO_EINVAL (count < 2, NULL fields). */
pico_status_t pico_pmr_finalize(pico_op_t op, const pico_accum_t* acc, double* var, void* stream);

/* lambda actually used in the normal equations (lambda * margin * lambda_max),
 * or 0 for lambda == 0.  Returns NAN for a NULL handle. */
double pico_lambda_abs(pico_op_t op);

/* Convergence monitor (Sec. 3.2.2 evaluation; Sec. 3.2.3 computes NRMSE on
 * standard-deviation maps): *nrmse = ||s - s_ref|| / ||s_ref|| with
 * s = sqrt(max(sum / count, 0)) from ``acc`` and s_ref = sqrt(max(ref_var, 0)),
 * ref_var device float64 [ny*nx].  Waits for ``stream``.  Reuses the
 * operator's scratch, so it must not overlap other calls on the same op.
 * Errors: PICO_EINVAL (NULL arguments, count < 1). */
pico_status_t pico_monitor_nrmse(pico_op_t op, const pico_accum_t* acc, const double* ref_var,
                                 double* nrmse, void* stream);

/* Reference-free error estimate of a running map, for adaptive stopping
 * (Sec. 5, Discussion: stopping on the per-voxel standard error): with m =
 * sum / N and s2 = (sumsq - N m^2) / (N - 1) the sample variance of the N
 * per-probe terms Re(conj v u), the estimate m has variance s2 / N, and the
 * std map sqrt(m) an error of about s2 / (4 N m) (first order); *proxy =
 * sqrt(sum_k s2_k / (4 N m_k) / sum_k m_k) over voxels with m_k > 0, the
 * expected NRMSE of the std map.  Needs acc->sumsq and count >= 2; waits for
 * ``stream``; reuses the operator's scratch (no overlap with other calls).
 *
 * pico_noise_map_adaptive adds probe tiles (probe_tile probes each, from
 * first_probe on) until *proxy <= target or max_probes probes are in; *used
 * and *proxy (either may be NULL) report where it stopped.  Same accumulator
 * and stats semantics as pico_noise_map; CG-SENSE operators only
 * (PICO_EUNSUPPORTED for CS).  Errors: PICO_EINVAL, PICO_EDEVICE, PICO_ENOTCONV. */
pico_status_t pico_monitor_stderr(pico_op_t op, const pico_accum_t* acc, double* proxy, void* stream);
pico_status_t pico_noise_map_adaptive(pico_op_t op, uint64_t seed, int64_t first_probe, int64_t max_probes,
                                      double target, int32_t dist, pico_accum_t* acc, pico_stats_t* stats,
                                      int64_t* used, double* proxy, void* stream);

/* Exact variance map diag(Sigma) into var (device float64 [ny*nx]) for a
 * phase-encode (PICO_CART_1D) operator: Sigma is block diagonal over image
 * columns (the mask is constant along kx), so the probe equal to 1 on one
 * image row of every column returns, on that row, the diagonal of every
 * column block; ny such probes give the whole map, exact up to the CG
 * tolerance (Sec. 2.1, Eqs. (8)-(10)).  Errors: PICO_EUNSUPPORTED for other
 * samplings, PICO_EINVAL, PICO_EDEVICE. */
pico_status_t pico_exact_diag(pico_op_t op, double* var, void* stream);

/* Reduced-resolution noise grid (Sec. 5, Discussion: noise maps follow the
 * smooth coil geometry and can be estimated on a coarser grid, then
 * interpolated back to the native one).
 *
 * pico_init_reduced builds the operator of the same acquisition restricted to
 * the central (ny/f) x (nx/f) block of k-space on an (ny/f) x (nx/f) grid:
 * coarse pixel m sits at native pixel f m (the centred DFT keeps pixel N/2 on
 * both grids), so the coarse maps are desc->maps at every f-th pixel, the
 * mask is its central block, and a non-Cartesian sample w (rad per native
 * pixel) is kept as f w when -pi/f <= w_y, w_x < pi/f.  Every other field of
 * desc (psi, lambda, CG, probe tile, storage, gridding) applies unchanged;
 * the handle works with every call of a CG-SENSE operator at the coarse size
 * (maps, accumulators and references are (ny/f) x (nx/f)).  The coarse map
 * estimates the native variance at the coarse pixels with no rescaling (unit
 * white k-space noise and orthonormal transforms keep the pixel level).
 * desc is read during the call only.  Errors: PICO_EINVAL (factor < 2, ny or
 * nx not divisible by f, an odd margin ny - ny/f or nx - nx/f, no sample in
 * the coarse band, or a coarse size the build does not cover),
 * PICO_EUNSUPPORTED (compressed-sensing reconstructions), PICO_ENOMEM,
 * PICO_EDEVICE.
 *
 * pico_upsample_map writes the native map var (device float64
 * [f ny_c][f nx_c]) from a coarse one (device float64 [ny_c][nx_c]) of a
 * reduced operator: native pixel (y, x) lies at coarse coordinate
 * (y / f, x / f), periodic bilinear weights (coarse values kept at the
 * coarse pixels).  Errors: PICO_EUNSUPPORTED (not a reduced operator),
 * PICO_EINVAL (NULL). */
pico_status_t pico_init_reduced(const pico_op_desc_t* desc, int32_t factor, void* stream, pico_op_t* out);
pico_status_t pico_upsample_map(pico_op_t coarse_op, const double* coarse, double* var, void* stream);

/* Kernel-class timing with HIP events recorded on the caller's stream.
 * pico_profile_start clears and enables recording; pico_profile_stop waits
 * for the recorded events and writes, per class k < PICO_PROF_KINDS, the
 * summed duration in ms and the launch count (either pointer may be NULL). */
enum {
  PICO_PROF_NORMAL_FIRST = 0,  /* first normal-operator application of a solve;
                                  CS: A^H w of the k-space probes               */
  PICO_PROF_NORMAL_ITER = 1,   /* x += alpha p, r -= alpha q, p = r + beta p
                                  fused with q = (M + lam) p and its dots;
                                  CS: q = M y of the tangents                   */
  PICO_PROF_CG_UPDATE = 2,     /* last x += alpha p of each solve               */
  PICO_PROF_CG_SCALARS = 3,    /* per-probe alpha / beta reductions             */
  PICO_PROF_ACCUM = 4,         /* FP64 accumulation of conj(v) u                */
  PICO_PROF_OTHER = 5,         /* Tikhonov middle product, PMR right-hand side;
                                  CS: gradient step, wavelets, threshold
                                  derivative and momentum of the tangents       */
  PICO_PROF_KINDS = 8
};
pico_status_t pico_profile_start(pico_op_t op);
pico_status_t pico_profile_stop(pico_op_t op, double* ms, int64_t* launches);

/* Pseudo multiple replica for a compressed-sensing operator (Sec. 1, App. C;
 * compared with the Jacobian probes in Sec. 3.2.3): replica r reconstructs
 * the perturbed whitened data b + sigma n_r, with n_r CN(0, I) on the
 * sampled k-space locations (Philox stream 1, element (c ny + ky) nx + kx,
 * draw r), by the same FP64 FISTA as the operator's own reconstruction x_0,
 * and adds d_r = (x_r - x_0) / sigma into acc: sum Re d, sum Im d, sum |d|^2
 * (all three buffers required; acc->count += nrep).  pico_pmr_finalize then
 * gives the unbiased sample variance, the replica estimate of diag(J J^H).
 * Replicas run min(probe_tile, 16) at a time; the first call allocates their
 * FP64 workspace.  Errors: PICO_EUNSUPPORTED for CG-SENSE operators (use
 * pico_pmr_baseline), PICO_EINVAL, PICO_ENOMEM, PICO_EDEVICE. */
pico_status_t pico_pmr_cs(pico_op_t op, uint64_t seed, int64_t first, int64_t nrep, double sigma,
                          pico_accum_t* acc, void* stream);

/* Gridding NUFFT data path of a PICO_NONCART operator built with kb_width > 0
 * (Sec. 3.2.2, 3.3; the reading of the gridding parameters is the one stated
 * at pico_op_desc_t.oversamp).  adjoint = 0: out[k][ncoils][nsamples] = A x
 * for x = in[k][ny][nx]; adjoint = 1: out[k][ny][nx] = A^H y for
 * y = in[k][ncoils][nsamples] (whitened coil samples).  complex64 device
 * arrays, 1 <= k <= probe_tile.  Uses the operator's scratch, so calls on one
 * operator must not overlap.  Errors: PICO_EUNSUPPORTED without a gridding
 * path, PICO_EINVAL, PICO_EDEVICE. */
pico_status_t pico_apply_nufft(pico_op_t op, int32_t adjoint, const void* in, void* out, int32_t k,
                               void* stream);

/* Tile-shape autotuner.  For the operator description desc (its device
 * arrays must be valid), times short noise-map runs (a warm-up tile, then at
 * least 2 tiles and 20 ms) of the candidates: probe_tile doubling from 16 to
 * 512 while its peak device bytes (pico_estimate_bytes) fit in max_bytes (0:
 * no limit) and the rate still grows by 3 % or more, for each phase-encode
 * normal form (column FFTs, dense FP32 blocks, split-FP16 blocks) of a
 * PICO_CART_1D CG-SENSE operator, with graph replay; then direct launches at
 * the fastest shape.  The fastest choice goes
 * to *out and, when cache_path is non-NULL, into that text file under a key
 * of the problem's shape (sampling, reconstruction, ny x nx, coils in buckets
 * of 8, CG iterations, Tikhonov or not, storage, FISTA / TV / wavelet
 * parameters, non-Cartesian samples in buckets of 4096).  A key already in the
 * file is returned without timing (out->from_cache = 1).  Every candidate
 * initialises its own operator (device memory from the allocator in effect);
 * synchronous on stream.  Errors: as pico_init; PICO_ENOMEM when no candidate
 * fits; PICO_EINVAL when the cache file cannot be written. */
typedef struct {
  int32_t probe_tile;           /* right-hand sides per batched solve / tangent batch */
  int32_t normal_form;          /* pico_op_desc_t.normal_form to use               */
  int32_t graph;                /* pico_op_desc_t.graph to use                     */
  double probes_per_s;          /* measured rate of the choice                     */
  int32_t from_cache;           /* 1: read from the cache file, not timed now      */
} pico_tune_t;
pico_status_t pico_autotune(const pico_op_desc_t* desc, uint64_t max_bytes, const char* cache_path, void* stream,
                            pico_tune_t* out);

/* Release the operator and its device memory (waits for its last stream). */
void pico_destroy(pico_op_t op);

/* Device memory of an operator, counted in 256-byte pieces: *resident is
 * what pico_init keeps after returning, *peak the most it holds during
 * pico_init (weight-builder and CS-primal temporaries).
 * pico_estimate_bytes computes both from the description alone (host only,
 * no device call; the same validation as pico_init, so PICO_EINVAL /
 * PICO_EUNSUPPORTED as there); pico_op_bytes reports what an initialised
 * operator actually took.  Either output pointer may be NULL. */
pico_status_t pico_estimate_bytes(const pico_op_desc_t* desc, uint64_t* resident, uint64_t* peak);
pico_status_t pico_op_bytes(pico_op_t op, uint64_t* resident, uint64_t* peak);

/* ------------------------------------------------------------------ serving
 * Many noise-map requests, each against its own operator, on the current
 * device (serving: HBM-budgeted admission, probe tiles of all admitted
 * requests in flight at once).
 *
 * pico_server_create takes one device allocation of hbm_budget bytes (rounded
 * down to 256) and starts a worker thread.  Every operator the server builds
 * lives in that allocation, so serving makes no further hipMalloc / hipFree.
 * A request is admitted in arrival order when one of max_slots slots is free
 * and either an idle resident operator has its key or its peak bytes
 * (pico_estimate_bytes) fit beside the resident operators (idle ones are
 * evicted, least recently used first, to make room); admitted requests each
 * have their own stream and up to tiles_in_flight probe tiles
 * (desc->probe_tile probes each) enqueued.  A finished request frees its slot
 * immediately; its operator stays resident, keyed by the content of the
 * description (scalar fields, psi, and a hash of the maps, mask, trajectory
 * and k-space data read on the device at admission), and a later request with
 * the same key runs on it without pico_init.  desc->probe_tile = 0 asks for
 * the tile shape of pico_server_set_tuning.
 *
 * A request adds probes [first_probe, first_probe + nprobes) into *acc
 * exactly as pico_noise_map(op, seed, first_probe, nprobes, dist, acc) on a
 * freshly initialised operator would (same tiles, same order, same values:
 * results do not depend on what else is being served).  acc->count is not
 * updated (the count is nprobes, reported back in the request info).
 *
 * Lifetimes: pico_server_submit copies the description and the host psi; the
 * device arrays it points to (maps, mask, traj, kdata) and the accumulator
 * buffers must stay valid until the request is reported done, and must be
 * ready when submitted (the server's streams do not wait on the caller's).
 *
 * Errors (synchronous, nothing queued): PICO_EINVAL / PICO_EUNSUPPORTED for a
 * description pico_init would reject or bad arguments, PICO_ENOMEM when the
 * request's peak bytes exceed the whole budget.  Errors found while serving
 * are reported per request in pico_request_info_t.status / .error.
 * Times are milliseconds on a steady clock since pico_server_create. */
typedef struct pico_server_s* pico_server_t;

typedef struct {
  uint64_t id;
  int32_t status;               /* pico_status_t of the request                 */
  int64_t first_probe, probes;
  double t_submit_ms, t_admit_ms, t_done_ms;
  uint64_t bytes_peak, bytes_resident;   /* estimate at submission             */
  int32_t probe_tile;           /* tile the request ran with                    */
  int32_t op_reused;            /* 1: served on a resident operator (no init)   */
  char error[160];              /* message when status != PICO_OK               */
} pico_request_info_t;

pico_status_t pico_server_create(uint64_t hbm_budget, int32_t max_slots, int32_t tiles_in_flight,
                                 pico_server_t* out);
pico_status_t pico_server_submit(pico_server_t srv, const pico_op_desc_t* desc, uint64_t seed,
                                 int64_t first_probe, int64_t nprobes, int32_t dist,
                                 const pico_accum_t* acc, uint64_t* req_id);
/* Moves up to max finished requests (oldest first) into out; *n = how many. */
pico_status_t pico_server_poll(pico_server_t srv, pico_request_info_t* out, int32_t max, int32_t* n);
/* Waits until every submitted request has finished (timeout_s < 0: no limit;
 * PICO_ENOTCONV if the timeout passes first). */
pico_status_t pico_server_wait_idle(pico_server_t srv, double timeout_s);
/* Budget, bytes handed out by the arena, queued and admitted request counts. */
pico_status_t pico_server_usage(pico_server_t srv, uint64_t* budget, uint64_t* arena_used,
                                int32_t* queued, int32_t* active);
/* Tile shapes for requests submitted with probe_tile = 0: read from the
 * autotuner's cache file at cache_path (pico_autotune; NULL or "" = none).
 * A request whose key is not in the file gets a power-of-two tile in 16..256
 * of about 2^23 voxels, and graph replay.  Errors: PICO_EINVAL (NULL server). */
pico_status_t pico_server_set_tuning(pico_server_t srv, const char* cache_path);
/* Resident operators kept between requests (busy or idle), their device
 * bytes, and how many admissions found an idle operator with the request's
 * key (hits) or built one (misses).  Any pointer may be NULL. */
pico_status_t pico_server_cache_stats(pico_server_t srv, int32_t* resident_ops, uint64_t* resident_bytes,
                                      int64_t* hits, int64_t* misses);
/* Serves everything already submitted, then stops the worker and frees the budget. */
void pico_server_destroy(pico_server_t srv);

/* Message for the last non-OK status on this thread ("" if none). */
const char* pico_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PICO_H_ */
