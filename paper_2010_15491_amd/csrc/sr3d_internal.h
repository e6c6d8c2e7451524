// Internal declarations shared by the libsr3d translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr3d.h"

namespace sr3d {

constexpr int kThreads = 256;      // threads per workgroup for every kernel here
constexpr int kMaxLen = 1024;      // largest FFT length supported
constexpr int kStencilVpt = 8;     // voxels per thread in the stencil kernels
constexpr int kStencilVox = kThreads * kStencilVpt;

// Device-side solver control block: the stop flag every predicated kernel
// reads, the iteration counter and the latest stopping-test values.
struct Ctrl {
  int done;       // 1 => all later predicated kernels return at once
  int iter;       // completed ADMM iterations
  int converged;  // tolerance test held
  int status;     // 0 or a negative sr3d_status found on the device
  int max_iter;
  int pad0;
  float tol, mu, lam, pad1;
  double primal_rel, dual_rel, objective;
  double inv_nl;  // 1 / N_l (LR Parseval factor of the data term)
};

// Unsigned 32-bit division by a runtime constant (round-up multiply method,
// Granlund & Montgomery 1994). Exact for 0 <= n < 2^31.
struct FastDiv {
  uint32_t d, m, s;
  FastDiv() : d(1), m(1), s(0) {}
  explicit FastDiv(uint32_t div) : d(div) {
    uint32_t l = 0;
    while ((1ull << l) < div) ++l;
    s = l;
    m = (uint32_t)((((1ull << 32) * ((1ull << l) - div)) / div) + 1);
  }
  __host__ __device__ inline uint32_t div(uint32_t n) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(n, m);
#else
    uint32_t t = (uint32_t)(((uint64_t)n * m) >> 32);
#endif
    return (t + n) >> s;
  }
};

// Per-stage HIP-event timing (SR3D_PROFILE). prof_begin/prof_end bracket a
// launch on its stream when the calling thread has profiling switched on.
enum Stage {
  kStFftR2cM, kStFftN, kStFftS, kStFold, kStIfftS, kStIfftN, kStIfftC2rM,
  kStStencilA, kStStencilB, kStReduce, kStSetup, kStCount
};
void prof_begin(int stage, hipStream_t st);
void prof_end(hipStream_t st);

bool fft_len_supported(int n);
// Device twiddle table exp(-2 pi i k / n), k < n, for the current device.
const float2 *twiddles(int n);
hipError_t ensure_device_tables();

// 3D transforms over a volume of S x N x M reals (m fastest). Half spectrum
// is S x N x (M/2+1) complex. `done` (device int, may be null) predicates
// every launch. The inverse overwrites `spec` and multiplies by `scale`.
hipError_t fft3d_forward(const float *in, float2 *spec, int S, int N, int M,
                         const int *done, hipStream_t st);
hipError_t fft3d_inverse(float2 *spec, float *out, int S, int N, int M, float scale,
                         const int *done, hipStream_t st);

// Fold / solve / unfold (eq. (8)-(12) and Algorithm 1 step 5a).
struct FoldArgs {
  const float2 *W;    // F Theta (TV) or F xbar (Tikhonov) half spectrum, or null
  const float2 *Lam;  // Lambda half spectrum
  const float2 *Yh;   // LR half spectrum of y
  float2 *X;          // output half spectrum (scaled by `scale`)
  const float *gm, *gn, *gs;  // |sigma(k)|^2 per axis (TV only)
  int S, N, M, Mh;
  int Sl, Nl, Ml, Mlh;
  int dr, dc, ds;
  int ml_eff;         // number of j_m values processed
  float cw;           // coefficient of W in B (mu or 2 lambda)
  float coefA;        // A = coefA * G (TV) or A = coefA (Tikhonov)
  int tv;
  float scale;        // 1 / N_h, folded into the output for the inverse FFT
  void *partial;      // data-term partial sums, one per workgroup (Acc), or null
  Ctrl *ctrl;
  const int *done;
};
int fold_blocks(const FoldArgs &a);
hipError_t fold_solve(const FoldArgs &a, bool fp64, hipStream_t st);

// Difference / shrink / dual kernels (Algorithm 1 steps 5b, 5c and the Theta
// of 5a). State nu = L x + d_prev holds (u, d): u = shrink(nu), d = nu - u.
struct StencilArgs {
  const float *x;
  float *nu;          // [3][N_h]
  float *theta;       // N_h: L^T (u - d)
  float *ltu;         // N_h: L^T u of the previous iteration (dual residual)
  int S, N, M;
  float thr;          // lambda / mu
  void *partA;        // [4][blocks] : |Lx-u'|^2, |Lx|^2, |u'|^2, sum |(Lx)_j|
  void *partB;        // [2][blocks] : |L^T(u'-u)|^2, |L^T d'|^2
  const int *done;
};
int stencil_blocks(int S, int N, int M);
// mode 0: iteration (nu <- L x + d(nu)); mode 1: init from x (nu <- L x);
// mode 2: init with x = 0 (nu <- 0).
hipError_t stencil_a(const StencilArgs &a, int mode, bool fp64, hipStream_t st);
// init != 0: first pass, no residual sums (ltu written only).
hipError_t stencil_b(const StencilArgs &a, int init, bool fp64, hipStream_t st);
// Final reduction of the partial sums and the stopping test.
hipError_t reduce_and_test(Ctrl *ctrl, const void *partA, int nbA, const void *partB, int nbB,
                           const void *partF, int nbF, bool fp64, hipStream_t st);

// Setup kernels.
hipError_t pad_psf(const float *psf, int Ks, int Kn, int Km, float *out, int S, int N, int M,
                   hipStream_t st);
hipError_t diff_tables(float *g, int S, int N, int M, hipStream_t st);  // g = [gm | gn | gs]
hipError_t ctrl_init(Ctrl *c, int max_iter, float tol, float mu, float lam, double inv_nl,
                     hipStream_t st);
hipError_t fill_zero(float *p, size_t n, hipStream_t st);
hipError_t spectrum_mul(float2 *W, const float2 *Lam, size_t n, float scale, hipStream_t st);
hipError_t decimate(const float *x, float *y, int S, int N, int M, int dr, int dc, int ds,
                    hipStream_t st);

}  // namespace sr3d
