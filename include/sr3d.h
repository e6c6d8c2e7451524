/*
 * sr3d.h -- C ABI of libsr3d, an MI355X (gfx950) implementation of the fast
 * Fourier-domain 3D single-image super-resolution solvers of Tuador et al.,
 * "A Novel Fast 3D Single Image Super-Resolution Algorithm" (arXiv 2010.15491).
 *
 * Problem (Sec. II-A, eq. (1)):  y = D H x + n
 *   x  HR volume of m_h x n_h x s_h voxels, y LR volume of m_l x n_l x s_l,
 *   H  circular blur by a PSF (eq. (2)), D decimation by d = dr*dc*ds keeping
 *      voxel offset 0 of every dr x dc x ds block.
 *
 * Memory layout of every volume: C order [s][n][m], m (rows) fastest -- the
 * lexicographic order of Sec. II-A. A PSF of Km x Kn x Ks taps is [Ks][Kn][Km];
 * its centre tap (K/2 per axis, integer division) is the origin of the
 * circular convolution. Half spectra (R2C output) are [s][n][m/2+1] complex
 * (interleaved float re, im), unnormalised.
 *
 * Ownership: the caller owns every pointer passed in (device memory unless
 * stated) and the workspace. The library owns only per-device twiddle tables
 * and the scratch of sr3d_tikhonov_noalloc (static device arrays, held until
 * the process ends) and a small pinned host block, created on first use and
 * released by sr3d_shutdown(). Inputs are read-only; outputs must not alias
 * inputs.
 *
 * Streams: all work is enqueued on the caller's stream. Functions return
 * after enqueueing, except sr3d_tv_admm / sr3d_batch, which synchronise the
 * stream to run the host stopping test and to fill `stats`.
 *
 * Errors: every function returns an sr3d_status. Argument errors are detected
 * on the host before any HIP call. Errors found on the device (Lambda(0) = 0
 * in a TV solve, a non-finite residual) are reported by sr3d_tv_admm /
 * sr3d_batch after their final synchronisation. sr3d_last_error() gives a
 * message for the calling thread's last failure.
 */
#ifndef SR3D_H
#define SR3D_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SR3D_OK = 0,
  SR3D_ERR_INVALID_ARG = -1,    /* NULL pointer, lambda/mu <= 0, tol < 0, max_iter < 1, rate < 1 */
  SR3D_ERR_NOT_DIVISIBLE = -2,  /* an HR dimension is not a multiple of its rate */
  SR3D_ERR_PSF_TOO_LARGE = -3,  /* a PSF extent exceeds the HR extent */
  SR3D_ERR_UNSUPPORTED_SIZE = -4, /* an FFT length (HR or LR) outside the supported set */
  SR3D_ERR_WORKSPACE = -5,      /* ws NULL or ws_bytes below sr3d_workspace_size() */
  SR3D_ERR_SINGULAR = -6,       /* Lambda(0) = 0: the TV x-update (Alg. 1 step 5a) is singular */
  SR3D_ERR_NONFINITE = -7,      /* a residual reduction produced NaN/Inf */
  SR3D_ERR_HIP = -8             /* a HIP runtime call failed (see sr3d_last_error) */
} sr3d_status;

typedef struct { int m, n, s; } sr3d_dims;   /* m fastest */
typedef struct { int dr, dc, ds; } sr3d_rate; /* decimation along m, n, s */

typedef struct {
  int iters;          /* ADMM iterations run (x-updates) */
  int converged;      /* 1 if the tolerance test held, 0 if max_iter was reached */
  double primal_rel;  /* ||Lx - u|| / max(||Lx||, ||u||) after the last iteration */
  double dual_rel;    /* mu ||L^T (u' - u)|| / (mu ||L^T d||) after the last iteration */
  double objective;   /* 1/2 ||y - DHx||^2 + lambda * sum_j ||(Lx)_j||_2 of the output x */
} sr3d_stats;

/* One TV super-resolution problem (Algorithm 1 of the paper, Sec. III-B). */
typedef struct {
  sr3d_dims hr;        /* HR size (m_h, n_h, s_h) */
  sr3d_rate rate;      /* (dr, dc, ds); LR size is hr / rate per axis */
  const float *y;      /* device, LR volume [s_l][n_l][m_l] */
  const float *psf;    /* device, PSF [Ks][Kn][Km] */
  sr3d_dims psf_dims;  /* (Km, Kn, Ks), each <= the HR extent */
  float lambda_tv;     /* lambda of eq. (3)/Algorithm 1 (TV weight), > 0 */
  float mu;            /* ADMM penalty mu > 0 */
  float tol;           /* relative primal/dual residual tolerance; 0 => run max_iter */
  int max_iter;        /* iteration cap, >= 1 */
  const float *x0;     /* device HR initial guess, or NULL for x0 = 0 */
  float *x;            /* device HR output [s_h][n_h][m_h] */
  float *state;        /* optional device buffer of 3*N_h floats, or NULL (see below) */
  float tol_dual;      /* tolerance of the relative dual residual; <= 0 means tol */
  float mu_data;       /* SR3D_DATA_L1 only: ADMM penalty of the data split, > 0 */
} sr3d_problem;

/* sr3d_problem.state: the ADMM state (u, d) is kept as nu = L x + d_prev
 * (three planes [3][s][n][m], components along m, n, s; with SR3D_REG_HAAR
 * one plane nu = W x + d_prev in the first N_h floats), from which
 * u = shrink(nu) and d = nu - u (Algorithm 1 steps 5b, 5c). If `state` is
 * non-NULL the solver keeps nu there instead of in the workspace, so the
 * final (u, d) can be read back; with SR3D_RESUME it also supplies the
 * initial state and x0 is ignored (checkpoint / resume). */

/* flags for sr3d_tv_admm / sr3d_batch */
#define SR3D_FP64_REDUCE 0x1   /* residual/objective reductions and the stopping test in FP64 (else FP32);
                                  per-voxel terms are FP32 and each thread first sums its
                                  own (at most 256 per stencil thread) in FP32 */
#define SR3D_RESUME      0x2   /* start from problem.state (must be non-NULL) */
#define SR3D_USE_GRAPH   0x4   /* replay captured iterations as a HIP graph */
#define SR3D_PROFILE     0x8   /* time every kernel launch with HIP events on the caller's
                                  stream; totals per stage via sr3d_profile_read (no graph) */
#define SR3D_WARM_DUAL   0x10  /* with x0: also start the scaled dual d from the minimum-norm
                                  solution of the x-update's stationarity at x0,
                                  mu L^T d = H^T D^T (y - D H x0) (nu0 = L(x0 + phi)) */
#define SR3D_UNFUSED     0x20  /* run the x-update as separate s-FFT, fold/solve and inverse
                                  s-FFT kernels even where the fused s-line kernel applies
                                  (same result up to FP32 rounding; for testing) */
#define SR3D_SEPARATE_R2C 0x40 /* with the fused x-update: run the stencil and the m-axis
                                  R2C of the next x-update as separate kernels even where the
                                  row length admits the fused stencil (64, 128, 192, 256);
                                  same bits, for testing */
#define SR3D_TV_ANISO    0x80  /* anisotropic TV, lambda sum_j ||(L x)_j||_1, instead of the
                                  isotropic sum_j ||(L x)_j||_2: one of the other regularisers
                                  the same x-step serves (Sec. III-B). Step 5b becomes a soft
                                  threshold of every component; the objective reports the l1
                                  form. Every other step is unchanged. */
#define SR3D_REG_HAAR    0x100000 /* regulariser lambda sum |detail coefficients of W x|, W the
                                  orthonormal 3D Haar transform with SR3D_HAAR_LEVELS levels
                                  (approximation coefficients not penalised): l1 in an orthogonal
                                  wavelet basis, another regulariser the same x-step serves
                                  (Sec. III-B). With W^T W = I, step 5a is the Tikhonov solve of
                                  eq. (12) with 2 lambda -> mu and xbar = W^T (u - d); steps 5b/5c
                                  act on the coefficients (soft threshold of the details). The
                                  state nu = W x + d is the first N_h floats of problem.state.
                                  Every HR dimension must be a multiple of 2^levels. Not with
                                  SR3D_TV_ANISO, SR3D_WARM_DUAL or sr3d_batch. */
#define SR3D_HAAR_LEVELS(j) (((j) & 0xf) << 16)  /* Haar levels for SR3D_REG_HAAR, 1..8 (0: 1) */
#define SR3D_DATA_L1     0x200000 /* l1 data term for non-Gaussian (impulsive, heavy-tailed)
                                  noise, which the paper's conclusion (Sec. V) names as future
                                  work: min ||D H x - y||_1 + lambda TV(x), by ADMM with a second
                                  split v = D H x - y (penalty problem.mu_data, scaled dual e).
                                  Step 5a is the x-step of Algorithm 1 with y -> y + v - e and
                                  mu -> mu / mu_data (unfused x-update); steps 5b/5c are
                                  unchanged (threshold lambda / mu); then
                                  v' = soft(D H x - y + e, 1 / mu_data), e' = e + D H x - y - v'.
                                  Initialisation applies both steps 5b/5c to x0 with zero duals.
                                  Stops when both splits' relative residuals meet the tolerances:
                                  the data split's primal |DHx - v' - y| / max(|DHx|, |v'|, |y|)
                                  and dual |H^T D^T (v' - v)| / |H^T D^T e'|; stats report the
                                  larger of the two splits' primal and dual, and the objective
                                  |DHx - y|_1 + lambda TV(x). Not with SR3D_REG_HAAR,
                                  SR3D_WARM_DUAL, SR3D_RESUME or sr3d_batch. */
#define SR3D_CHECK_INTERVAL(k) (((k) & 0xff) << 8)  /* host polls the device stop flag every k iterations (default 8) */

/* operations for sr3d_workspace_size */
#define SR3D_OP_TIKHONOV 1
#define SR3D_OP_TV_ADMM  2
#define SR3D_OP_BATCH    3
#define SR3D_OP_DEGRADE  4
#define SR3D_OP_FFT      5
#define SR3D_OP_PSF_FIT  6
#define SR3D_OP_TIKHONOV_MF 7  /* count = number of frames */
#define SR3D_OP_TV_ADMM_MF  8  /* count = number of frames */

/* Workspace bytes needed by `op` for problem(s) p[0..count-1] (count = 1
 * except for SR3D_OP_BATCH). Only hr, rate and psf_dims are read. Returns 0
 * for invalid sizes. For SR3D_OP_FFT, p->hr gives the transform size. */
size_t sr3d_workspace_size(int op, const sr3d_problem *p, int count);

/* 3D-FSR-l2-l2: x = argmin 1/2||y - DHx||^2 + lambda ||x - xbar||^2, the
 * closed form of eq. (12) (Sec. III-A): one 3D R2C FFT, a pointwise solve per
 * alias group (eq. (8)-(12)), one 3D C2R FFT.
 *   y     device LR volume, xbar device HR volume or NULL (xbar = 0),
 *   lambda > 0 (eq. (5)), x device HR output. */
int sr3d_tikhonov(sr3d_dims hr, sr3d_rate rate, const float *y, const float *psf,
                  sr3d_dims psf_dims, const float *xbar, float lambda, float *x,
                  void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as sr3d_tikhonov, through the same kernels and with the same result
 * bits, with no workspace argument. Its workspace is a static device array
 * of SR3D_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the library runs on
 * holds until the process ends; the call allocates nothing. A problem whose
 * sr3d_workspace_size(SR3D_OP_TIKHONOV, ...) exceeds the array (e.g. more
 * than a 128^3 HR volume) returns SR3D_ERR_WORKSPACE before any HIP call.
 * The first call on a device looks up the array's address and uploads the
 * FFT twiddle tables with a synchronous copy, so make it before any graph
 * capture; later calls only enqueue kernels on `stream`. Every call on one
 * GPU uses that GPU's one array, whose contents persist between calls (no
 * part of it needs clearing: each buffer is written before it is read):
 * calls that overlap on one GPU (other streams, other threads) race. */
#define SR3D_NOALLOC_SCRATCH_BYTES (64u << 20)
int sr3d_tikhonov_noalloc(sr3d_dims hr, sr3d_rate rate, const float *y, const float *psf,
                          sr3d_dims psf_dims, const float *xbar, float lambda, float *x,
                          hipStream_t stream);

/* 3D-FSR-l2-TV: Algorithm 1 (Sec. III-B). Initialisation u0, d0 from x0 by
 * steps 5b/5c with d = 0 (x0 = 0 gives u0 = d0 = 0). Each iteration runs the
 * x-update 5a through eq. (12) in the Fourier domain (the zero-frequency alias
 * group, where Gamma = 1/G is unbounded, by exact elimination), then 5b, 5c.
 * Stops when ||Lx-u'|| <= tol max(||Lx||,||u'||) and
 * mu||L^T(u'-u)|| <= tol_dual mu||L^T d'|| (tol_dual = tol unless set), or
 * after max_iter iterations. The flags SR3D_TV_ANISO and SR3D_REG_HAAR
 * select the other regularisers the same x-step serves; with SR3D_REG_HAAR,
 * L is the Haar transform W in everything above.
 * `stats` (host) may be NULL. */
int sr3d_tv_admm(const sr3d_problem *p, int flags, sr3d_stats *stats,
                 void *ws, size_t ws_bytes, hipStream_t stream);

/* 3D multi-frame SR (named as future work in Sec. V): nframes (1..4) LR
 * volumes y[f] of the same HR volume, frame f observed after a circular
 * shift of the HR grid by shifts[3 f + (0, 1, 2)] = (t_m, t_n, t_s) voxels:
 * y_f = D S_f H x + n_f with (S_f z)[i] = z[i + t_f]. Because a shift is a
 * phase factor in the Fourier domain, eq. (8) still splits the normal
 * equations into one d x d system per alias group, with one rank-one term
 * per frame; it is solved in FP64 through an F x F Woodbury system (and the
 * zero-frequency group of a TV solve by a Schur complement). y is a host
 * array of device pointers, shifts a host array; d must be 1, 2, 4, 8, 16 or
 * 32. Workspace: sr3d_workspace_size(SR3D_OP_TIKHONOV_MF or
 * SR3D_OP_TV_ADMM_MF, p, nframes).
 * sr3d_tikhonov_mf: min sum_f 1/2 ||y_f - D S_f H x||^2 + lambda ||x - xbar||^2.
 * sr3d_tv_admm_mf: Algorithm 1 with the data term sum_f 1/2 ||y_f - D S_f H x||^2
 * (problem.y is not read; the unfused x-update and the tiled stencil run);
 * the flags of sr3d_tv_admm except SR3D_REG_HAAR, SR3D_WARM_DUAL and
 * SR3D_DATA_L1. The objective reports the multi-frame data term. */
int sr3d_tikhonov_mf(sr3d_dims hr, sr3d_rate rate, int nframes, const float *const *y,
                     const int *shifts, const float *psf, sr3d_dims psf_dims, const float *xbar,
                     float lambda, float *x, void *ws, size_t ws_bytes, hipStream_t stream);
int sr3d_tv_admm_mf(const sr3d_problem *p, int nframes, const float *const *y, const int *shifts,
                    int flags, sr3d_stats *stats, void *ws, size_t ws_bytes, hipStream_t stream);

/* Many independent TV problems p[0..count-1] of uneven sizes and rates,
 * solved together: each stage of an iteration is one launch over all active
 * volumes; converged volumes drop out on the device. stats: host array of
 * `count` entries or NULL. */
int sr3d_batch(const sr3d_problem *p, int count, int flags, sr3d_stats *stats,
               void *ws, size_t ws_bytes, hipStream_t stream);

/* PSF estimation (Sec. IV-B: the PSF of the real data is a fitted 3D
 * Gaussian). From an HR reference x (e.g. a micro-CT registered to the LR
 * grid) and the LR volume y, fits sigma = (sigma_m, sigma_n, sigma_s) of a
 * separable Gaussian sampled on 2 radius[a] + 1 taps per axis and normalised
 * to sum 1, with an intensity gain and offset:
 *   min 1/2 ||y - gain D H_sigma x - offset||^2,
 * by Levenberg-Marquardt steps on the Gauss-Newton model; each step is one
 * pass over the spectrum of x (eq. (8): the LR spectrum of D H_sigma x is
 * the alias-group mean of Lambda X). The offset only moves the zero
 * frequency and is solved exactly. Starts from sigma0 and the least-squares
 * gain for it; stops when a step changes no parameter by more than `tol`
 * relative (FP32 data fix the minimiser to about 1e-7 relative, so 1e-6 is
 * a natural choice), or after max_iter steps. x HR and y LR device volumes; res
 * (host) receives the fit; the call synchronises `stream`. */
typedef struct {
  double sigma[3];   /* (sigma_m, sigma_n, sigma_s) */
  double gain, offset;
  double objective;  /* 1/2 ||y - gain D H_sigma x - offset||^2 at the fit */
  int passes;        /* passes over the spectrum */
  int converged;     /* 1 if the step tolerance was met */
} sr3d_psf_fit_result;
int sr3d_psf_fit(sr3d_dims hr, sr3d_rate rate, const float *x, const float *y, const int radius[3],
                 const double sigma0[3], int max_iter, double tol, sr3d_psf_fit_result *res,
                 void *ws, size_t ws_bytes, hipStream_t stream);

/* Forward model of eq. (1) without noise: y = D H x (circular blur by the
 * PSF, then decimation). x device HR, y device LR. */
int sr3d_degrade(sr3d_dims hr, sr3d_rate rate, const float *x, const float *psf,
                 sr3d_dims psf_dims, float *y, void *ws, size_t ws_bytes,
                 hipStream_t stream);

/* Unnormalised 3D R2C DFT of a real volume [s][n][m] into its half spectrum
 * [s][n][m/2+1] (complex interleaved), and the inverse C2R (scaled by 1/N, so
 * that sr3d_irfft3d(sr3d_rfft3d(v)) = v). The inverse overwrites `spec`. */
int sr3d_rfft3d(sr3d_dims dims, const float *in, float *spec, hipStream_t stream);
int sr3d_irfft3d(sr3d_dims dims, float *spec, float *out, hipStream_t stream);

/* Learned warm start (not in the paper): x0 = x + f(x) for Algorithm 1,
 * where x is the Tikhonov solution (eq. (12)) and f a 3D CNN of six 3x3x3
 * convolutions (1->32, four 32->32, 32->1 channels) with bias, ReLU after the
 * first five and periodic padding. Tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) for
 * offsets along (s, n, m); conv(a)[v][co] = sum_t sum_ci W[t][co][ci]
 * a[v + off_t][ci] + b[co]. Parameters are one FP32 vector: per layer W as
 * [27][cout][cin] then b[cout]. Weights and hidden activations are rounded to
 * bfloat16 (nearest even; hidden activations stored channels-last,
 * [voxel][32]); sums accumulate in FP32 on BF16 matrix cores. Loss: mean
 * squared error against a target volume; optimiser: Adam on the FP32
 * parameters. All pointers are device memory owned by the caller. */
size_t sr3d_cnn_param_count(void);
/* He-uniform weights (last layer scaled by 0.1), zero biases, from a
 * counter-based generator (SplitMix64) seeded with `seed`. */
int sr3d_cnn_init(float *params, unsigned long long seed, hipStream_t stream);
/* Workspace for sr3d_cnn_forward (training = 0) or sr3d_cnn_grad (training = 1)
 * on a volume of size dims. */
size_t sr3d_cnn_workspace_size(sr3d_dims dims, int training);
/* y = x + f(x); x, y HR volumes [s][n][m] (may not alias). */
int sr3d_cnn_forward(sr3d_dims dims, const float *params, const float *x, float *y,
                     void *ws, size_t ws_bytes, hipStream_t stream);
/* loss (device float) = mean((x + f(x) - target)^2) and grad (device,
 * sr3d_cnn_param_count() floats) = its gradient with respect to params. */
int sr3d_cnn_grad(sr3d_dims dims, const float *params, const float *x, const float *target,
                  float *grad, float *loss, void *ws, size_t ws_bytes, hipStream_t stream);
/* One Adam step (bias-corrected, step counted from 1) on all parameters. */
int sr3d_cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                  float beta1, float beta2, float eps, hipStream_t stream);
/* Single convolution layers (the network's building blocks). Forward:
 * cin = 1, cout = 32 reads the FP32 volume x (rounded to bfloat16);
 * cin = cout = 32 reads in_bf16 [voxel][32]. weight [27][cout][cin] FP32
 * (rounded to bfloat16), bias [cout]; output after ReLU as bfloat16
 * [voxel][32] and, if out_f32 is non-NULL, before rounding in FP32.
 * Backward (cin = cout = 32): gweight [27][32][32] then gbias [32] (FP32)
 * from the layer input act_in_bf16 and the output gradient gout_bf16; if
 * gin_bf16 is non-NULL also the input gradient, zeroed where mask_bf16 <= 0. */
size_t sr3d_conv3d_workspace_size(sr3d_dims dims);
int sr3d_conv3d_forward(sr3d_dims dims, int cin, int cout, const void *in_bf16, const float *x,
                        const float *weight, const float *bias, void *out_bf16, float *out_f32,
                        void *ws, size_t ws_bytes, hipStream_t stream);
int sr3d_conv3d_backward(sr3d_dims dims, const void *act_in_bf16, const void *gout_bf16,
                         const float *weight, const void *mask_bf16, void *gin_bf16,
                         float *gin_f32, float *gweight, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* FFT autotuner. Every axis kernel (R2C/C2R along m, forward/inverse along n
 * and s) comes in tile variants of 2048, 4096 and 8192 complex elements per
 * workgroup. sr3d_autotune times each variant for every HR and LR transform
 * that problems p[0..count-1] need and keeps the fastest per (axis kind,
 * length) for all later calls on this process; lengths already tuned are
 * skipped unless `force` is non-zero. It allocates scratch device memory,
 * synchronises `stream`, and must not run under graph capture. The choices
 * can be written to and read from a text file (one "kind length variant" per
 * line). Untuned lengths use the 4096-element tile. */
int sr3d_autotune(const sr3d_problem *p, int count, int force, hipStream_t stream);
int sr3d_tune_save(const char *path);
/* Returns the number of entries read, or SR3D_ERR_INVALID_ARG if the file
 * cannot be opened. */
int sr3d_tune_load(const char *path);

/* Per-stage kernel timing gathered by calls made with SR3D_PROFILE (a
 * tracing aid). Stage indices run from 0 while the call returns SR3D_OK;
 * past the last stage it returns SR3D_ERR_INVALID_ARG. *name is a static
 * string, *total_ms the summed HIP-event time of the stage's launches and
 * *launches their count. Any output pointer may be NULL. */
int sr3d_profile_read(int stage, const char **name, double *total_ms, long *launches);
/* Clears the per-stage totals. */
void sr3d_profile_reset(void);
/* Restricts SR3D_PROFILE timing to the stages whose bit is set (bit i is
 * stage index i of sr3d_profile_read); ~0u, the initial value, times every
 * stage. Each timed launch adds two event records to the stream, so timing
 * one stage disturbs a run less than timing all of them. Process-wide. */
void sr3d_profile_select(unsigned stage_mask);

/* Human-readable name of a status code. */
const char *sr3d_status_string(int status);
/* Message describing the calling thread's last failed call ("" if none). */
const char *sr3d_last_error(void);
/* Releases the host staging and forgets the per-device table addresses (the
 * static device arrays themselves stay until the process ends). */
void sr3d_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* SR3D_H */
