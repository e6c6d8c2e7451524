// Internal declarations shared by the libsr3d translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sr3d.h"

namespace sr3d {

constexpr int kThreads = 256;      // threads per workgroup for every kernel here
constexpr int kMaxLen = 1024;      // largest FFT length supported

// Device-side solver control block: the stop flag every predicated kernel
// reads, the iteration counter and the latest stopping-test values.
struct Ctrl {
  int done;       // 1 => all later predicated kernels return at once
  int iter;       // completed ADMM iterations
  int converged;  // tolerance test held
  int status;     // 0 or a negative sr3d_status found on the device
  int max_iter;
  int counted;    // batch: this volume's stop has been counted
  float tol, mu, lam, tol_dual;
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
  kStStencil, kStReduce, kStSolveS, kStStencilR2c, kStWavelet, kStSetup, kStL1Data, kStCount
};
void prof_begin(int stage, hipStream_t st);
void prof_end(hipStream_t st);

#define SR3D_FFT_LENGTHS(X) \
  X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
  X(384) X(512) X(768) X(1024)

bool fft_len_supported(int n);

// Axis kernels and their tile variants (fft_m.hip, fft_strided.hip). A
// descriptor holds one volume's arguments; batch launches take an array of
// descriptors and a list of (volume, tile) items, one workgroup per item.
// Final reduction and stopping test of an iteration, run by one extra
// workgroup of another launch (ctrl == nullptr: none).
struct RedArgs {
  Ctrl *ctrl;
  const void *ps;  // stencil partials [6][nbs]
  int nbs;
  const void *pf;  // data-term partials [nbf]
  int nbf;
  int fp64;        // partials are double (else float)
};
struct StridedDesc {
  float2 *data;
  int ncols;
  FastDiv inner;
  int inner_valid;  // columns with (c mod inner) >= inner_valid are row padding: skipped
  long outer_stride, estride;
  const int *done;
  RedArgs red;  // single-volume launches: a reduction run by one extra workgroup
};
inline StridedDesc make_strided_desc(float2 *data, long ncols, long inner, long outer_stride,
                                     long estride, const int *done, long inner_valid = -1) {
  StridedDesc d;
  d.data = data;
  d.ncols = (int)ncols;
  d.inner = FastDiv((uint32_t)inner);
  d.inner_valid = (int)(inner_valid < 0 ? inner : inner_valid);
  d.outer_stride = outer_stride;
  d.estride = estride;
  d.done = done;
  d.red = RedArgs{};
  return d;
}
struct RowDesc {
  const float *rin;  // R2C input rows
  float2 *spec;      // half-spectrum rows (R2C output / C2R input)
  float *rout;       // C2R output rows
  long nrows;
  float scale;       // C2R output scale
  const int *done;
  // Column order of the stored half spectrum (even M only): kofp[p] is the
  // frequency k_m held at position p, posk its inverse. Null: natural order.
  const int *kofp, *posk;
  int pitch;  // complex entries between spectrum rows (0: M/2 + 1)
  RedArgs red;  // R2C: the previous iteration's final reduction, in one extra workgroup
};
int strided_tiles(int L, int v, long ncols);
int row_tiles(int M, int v, long nrows);
hipError_t launch_strided_batch(int L, bool inv, int v, const StridedDesc *descs, const int2 *items,
                                int nitems, hipStream_t st);
hipError_t launch_rows_batch(int M, bool c2r, int v, const RowDesc *descs, const int2 *items,
                             int nitems, hipStream_t st);
enum FftKind { kFftR2cM, kFftC2rM, kFftFwdN, kFftInvN, kFftFwdS, kFftInvS, kFftKinds };
hipError_t launch_r2c_m_v(const float *in, float2 *out, long nrows, int M, int v, const int *done,
                          hipStream_t st, const int *kofp = nullptr, const int *posk = nullptr,
                          int pitch = 0, const RedArgs *red = nullptr);
hipError_t launch_c2r_m_v(const float2 *in, float *out, long nrows, int M, float scale, int v,
                          const int *done, hipStream_t st, const int *kofp = nullptr,
                          const int *posk = nullptr, int pitch = 0);
hipError_t launch_strided_v(float2 *data, int L, long ncols, long inner, long outer_stride,
                            long estride, bool inv, int v, const int *done, hipStream_t st,
                            long inner_valid = -1, const RedArgs *red = nullptr);
int fft_variant(int kind, int len);
void fft_set_variant(int kind, int len, int v);
// Times every tile variant of every axis kernel a volume S x N x M uses and
// keeps the fastest (skips lengths already tuned unless force). Allocates
// scratch with hipMalloc (up to 8 volume-sized buffers, at least 640 MiB
// together, rotated so timings include HBM traffic) and synchronises the
// stream.
// pitch: row pitch the m and n kinds are timed with (0: natural layout).
hipError_t fft_autotune(int S, int N, int M, int pitch, bool force, hipStream_t st);
int fft_tune_save(const char *path);
int fft_tune_load(const char *path);
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
// The forward transform of K volumes stored back to back (inputs S N M
// floats apart, spectra S N (M/2+1) apart), one launch per axis.
hipError_t fft3d_forward_stack(const float *in, float2 *spec, int K, int S, int N, int M,
                               const int *done, hipStream_t st);
// The m and n passes alone (the s axis is left to the fused x-update), with
// the m columns stored in the order kofp / posk and rows `pitch` apart.
hipError_t fft2d_mn_forward(const float *in, float2 *spec, int S, int N, int M, const int *kofp,
                            const int *posk, int pitch, const int *done, hipStream_t st,
                            const RedArgs *red = nullptr);
hipError_t fft2d_mn_inverse(float2 *spec, float *out, int S, int N, int M, float scale,
                            const int *kofp, const int *posk, int pitch, const int *done,
                            hipStream_t st);
// The n pass alone, forward, over a spectrum whose m pass is done. With `red`
// (N > 1), one extra workgroup runs that reduction.
hipError_t fft_n_forward(float2 *spec, int S, int N, int M, int pitch, const int *done,
                         hipStream_t st, const RedArgs *red = nullptr);

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
  float2 *dhx;        // LR half spectrum of D H x for the new x (unscaled), or null
};
int fold_blocks(const FoldArgs &a);

// Multi-frame fold / solve / unfold (fold_mf.hip): F LR frames of HR-shifted
// copies, y_f = D S_f H x + n_f, (S_f z)[i] = z[i + t_f].
constexpr int kMaxFrames = 4;
struct MfArgs {
  const float2 *W;    // F Theta (TV) or F xbar (Tikhonov) half spectrum, or null
  const float2 *Lam;  // Lambda half spectrum
  const float2 *Yf;   // the frames' LR half spectra, nlspec apart
  long nlspec;
  float2 *X;          // output half spectrum (scaled by `scale`)
  const float *gm, *gn, *gs;
  const float2 *twm, *twn, *tws;  // exp(-2 pi i k / n) for n = M, N, S
  int t[kMaxFrames][3];           // shifts (t_m, t_n, t_s) of the frames
  float2 r[kMaxFrames][32];       // member phase exp(2 pi i (a t_m/d_r + b t_n/d_c + c t_s/d_s)),
                                  // member q = (c d_c + b) d_r + a
  int F;
  int S, N, M, Mh, Sl, Nl, Ml, Mlh, dr, dc, ds, ml_eff;
  float cw, coefA;
  int tv;
  float scale;
  void *partial;      // data-term partial sums, one per workgroup (Acc), or null
  Ctrl *ctrl;
  const int *done;
};
bool fold_mf_supported(int d, int nframes);
int fold_mf_blocks(const MfArgs &a);
hipError_t fold_solve_mf(const MfArgs &a, bool fp64, hipStream_t st);
hipError_t fold_solve(const FoldArgs &a, bool fp64, hipStream_t st);
hipError_t dual_init_spectrum(const FoldArgs &a, hipStream_t st);
hipError_t fold_solve_batch(int D, const FoldArgs *descs, const int2 *items, int nitems, bool fp64,
                            hipStream_t st);

// Fused x-update along s (solve_s.hip): one workgroup loads every s-line of
// a set of (k_n, k_m) columns closed under aliasing and conjugation, does the
// forward s-FFT, solves every alias group of those columns, does the inverse
// s-FFT and writes the lines back. See SolveSPlan for the unit structure.
struct SolveSArgs {
  float2 *W;          // S x N x Mh spectrum after the m and n passes (m columns
                      // in plan order); overwritten with the scaled x-update
  const float2 *Lg;   // Lambda per (unit, member, slot)
  const float2 *Yg;   // LR spectrum of y per (unit, slot)
  const int *tab;     // plan tables (see SolveSPlan)
  const float *gm, *gn, *gs;
  int S, N, M, Mh, Sl, Nl, Ml;
  int P;              // row pitch of W (complex entries)
  int dr, dc, ds, D;
  int NG, NB, CB, gmax, units;
  int o_p0, o_cnt, o_mj, o_nj;
  float mu, scale;
  void *partial;      // data-term partial sums, one per unit (Acc)
  Ctrl *ctrl;
  const int *done;
  int a_pos;          // A > 0 at every member (A = mu with gm = 1, gn = gs = 0: the Tikhonov
                      // x-step of the wavelet form); else A(0) = 0 and the zero-frequency
                      // group is eliminated exactly
  float2 *dhx;        // optional: the LR half spectrum (S_l x N_l x (M_l/2 + 1)) of D H x
                      // of the new x, written at every stored entry
};
// Unit structure. The LR columns (j_n, j_m) are split into n-groups (one
// class {j_n, -j_n}, or the two self-conjugate classes {0} and {N_l/2}) and
// m-blocks (CB consecutive classes {j_m, -j_m}); a unit is (n-group, m-block).
// Its lines are the stored columns (k_n, k_m) with k_n mod N_l in the n-group
// and k_m mod M_l in the m-block: every alias member of every group of the
// unit, or its conjugate mirror, lies on one of them, and no other unit reads
// or writes them. The m columns of a class are stored next to each other
// (position order kofp), so each m-block is one contiguous run per row.
struct SolveSPlan {
  bool fused;   // the fused kernel handles this geometry
  int dm;       // member-array bound of the kernel instance (8, 16 or 32)
  int pitch;    // row pitch of the spectrum (Mh rounded up to 16 for long rows)
  int NG, NB, CB, units, gmax;
  int o_p0, o_cnt, o_mj, o_nj;
  // Host image of the device table:
  //   kofp[Mh] | posk[Mh] | p0[NB] | cnt[NB] | mj[NB*CB] | nj[NG*2]
  std::vector<int> tab;
};
// Plans the fused x-update for an S x N x M volume at rates (dr, dc, ds).
SolveSPlan solve_s_plan(int S, int N, int M, int dr, int dc, int ds);
// Y alone in unit order (the l1 data term changes y' every iteration).
hipError_t solve_s_gather_y(const SolveSArgs &a, const float2 *yh, int Mlh, hipStream_t st);
hipError_t solve_s_gather(const SolveSArgs &a, const float2 *lam, const float2 *yh, int Mlh,
                          hipStream_t st);
// descs: device array of per-volume arguments; items: (volume, unit) per
// workgroup, or null for one volume (descs[0]) with `units` workgroups.
// gr: the m and n rate every volume of the launch shares, where an instance is
// specialised for it (2 at member bounds 8 and 16, 4 at 32), else 0.
hipError_t solve_s(int S, int dm, int d, int gr, const SolveSArgs *descs, const int2 *items,
                   int nwg, bool fp64, hipStream_t st);

// Fused difference / shrink / dual / Theta pass (Algorithm 1 steps 5b, 5c and
// the Theta of the next 5a). State nu = L x + d_prev holds (u, d):
// u = shrink(nu), d = nu - u.
struct AdmmStencilArgs {
  const float *x;      // HR volume, or null for x = 0
  const float *nu_in;  // [3][N_h] state before the step, or null (initialisation: d = 0)
  float *nu_out;       // [3][N_h] state after the step (must not alias nu_in)
  float *theta;        // N_h: L^T (u' - d')
  int S, N, M;
  float thr;           // lambda / mu
  void *part;          // [6][blocks]: |Lx-u'|^2, |Lx|^2, |u'|^2, sum|(Lx)_j|, |L^T(u'-u)|^2, |L^T d'|^2
  const int *done;
  int aniso;           // anisotropic TV: per-component shrink, |(Lx)_j|_1 in the objective
};
struct StencilPlan {
  int tiles_m, tiles_n, chunks, L, blocks;
};
StencilPlan stencil_plan(int S, int N, int M);
hipError_t admm_stencil(const AdmmStencilArgs &a, bool stats, bool fp64, hipStream_t st);
// The stencil with the next x-update's m-axis R2C of Theta fused in
// (stencil_r2c.hip): writes the half spectrum of Theta (positions in the
// order kofp, rows `pitch` apart) instead of Theta. a.x and a.nu_in must be
// non-null; the residual sums are always formed.
bool stencil_r2c_supported(int M);
// The fused stencil handles this volume: a supported row length, and every
// state and spectrum offset within 32 bits.
bool stencil_r2c_fits(int S, int N, int M, int pitch);
StencilPlan stencil_r2c_plan(int S, int N, int M);
hipError_t admm_stencil_r2c(const AdmmStencilArgs &a, float2 *spec, const int *kofp, int pitch,
                            bool fp64, hipStream_t st);
struct BatchStencilDesc {
  AdmmStencilArgs a;
  float *nu[2];
  StencilPlan pl;      // tiled plan, or stencil_r2c_plan for the fused stencil
  float2 *spec;        // fused stencil: the x-update's spectrum (kofp order,
  const int *kofp;     // rows `pitch` apart)
  int pitch;
};
// The fused stencil over (volume, tile) items of volumes with row length M.
hipError_t admm_stencil_r2c_batch(int M, const BatchStencilDesc *descs, const int2 *items,
                                  int nitems, int k, bool fp64, bool aniso, hipStream_t st);
hipError_t admm_stencil_batch(const BatchStencilDesc *descs, const int2 *items, int nitems, int k,
                              bool fp64, bool aniso, hipStream_t st);
hipError_t theta_from_nu(const float *nu, float *theta, int S, int N, int M, float thr,
                         bool aniso, hipStream_t st);
// Final reduction of the partial sums and the stopping test.
hipError_t reduce_and_test(Ctrl *ctrl, const void *partS, int nbS, const void *partF, int nbF,
                           bool fp64, hipStream_t st);
struct ReduceDesc {
  Ctrl *ctrl;
  const void *ps;
  int nbs;
  const void *pf;
  int nbf;
};
hipError_t reduce_and_test_batch(const ReduceDesc *descs, int nvol, int *active, bool fp64,
                                 hipStream_t st);

// l1 data term (l1data.hip): LR-grid steps of the second split v = D H x - y.
hipError_t l1_weights(const float2 *lam, float *w, int S, int N, int M, int dr, int dc, int ds,
                      hipStream_t st);
int l1_blocks(long n);
hipError_t l1_update(const float *t, const float *y, float *v, float *e, float *yp, float *dv,
                     long n, float thr, bool init, void *part, bool fp64, const int *done,
                     hipStream_t st);
hipError_t l1_wnorm(const float2 *A, const float2 *B, const float *w, long n, void *part, bool fp64,
                    const int *done, hipStream_t st);
hipError_t l1_reduce_test(Ctrl *c, const void *ps, int nbs, const void *pl, int nbl, const void *pw,
                          int nbw, bool fp64, hipStream_t st);

// PSF estimation (psf_fit.hip): one Gauss-Newton pass over the HR half
// spectrum X of the reference with per-axis kernel tables (l_m | l_n | l_s |
// dl_m | dl_n | dl_s), leaving psf_fit_nsums() FP64 totals in `out`.
int psf_fit_blocks(long nlspec);
int psf_fit_nsums();
hipError_t psf_fit_sums(const float2 *X, const float2 *Yh, const float *tab, float alpha, int S,
                        int N, int M, int dr, int dc, int ds, double *part, double *out,
                        hipStream_t st);

// Setup kernels.
hipError_t pad_psf(const float *psf, int Ks, int Kn, int Km, float *out, int S, int N, int M,
                   hipStream_t st);
hipError_t diff_tables(float *g, int S, int N, int M, hipStream_t st);  // g = [gm | gn | gs]
hipError_t ctrl_init(Ctrl *c, int max_iter, float tol, float tol_dual, float mu, float lam,
                     double inv_nl, hipStream_t st);
hipError_t fill_zero(float *p, size_t n, hipStream_t st);

// l1 of orthonormal 3D Haar details through the same x-step (haar.hip).
// haar3: `levels` levels of W (or W^T with `inverse`) of an S x N x M volume,
// every dimension a multiple of 2^levels; the forward transform reads `in`
// and works in place on `out`, the inverse works in place on `out`.
hipError_t haar3(const float *in, float *out, int S, int N, int M, int levels, bool inverse,
                 const int *done, hipStream_t st);
// Steps 5b/5c on coefficients cz = W x, overwritten by u' - d'. mode 0: from
// the state nu_in, residual sums into part ([6][wavelet_blocks]); 1: from cz
// with d_prev = 0 (initialisation); 2: cz = u - d of the state nu_in alone.
hipError_t wavelet_admm(float *cz, const float *nu_in, float *nu_out, int S, int N, int M,
                        int levels, float thr, int mode, void *part, bool fp64, const int *done,
                        hipStream_t st);
int wavelet_blocks(int S, int N, int M);
// W, steps 5b/5c and W^T in one pass for levels <= 3 (modes as wavelet_admm):
// reads x (mode 0, 1; null in mode 1 means x = 0) and nu_in (mode 0, 2),
// writes nu_out (mode 0, 1) and xbar; residual sums into part
// ([6][wavelet_fused_blocks]) in mode 0.
hipError_t wavelet_fused(const float *x, const float *nu_in, float *nu_out, float *xbar, int S,
                         int N, int M, int levels, float thr, int mode, void *part, bool fp64,
                         const int *done, hipStream_t st);
int wavelet_fused_blocks(int S, int N, int M, int levels);
hipError_t add_to(float *y, const float *x, size_t n, hipStream_t st);
hipError_t spectrum_mul(float2 *W, const float2 *Lam, size_t n, float scale, hipStream_t st);
hipError_t decimate(const float *x, float *y, int S, int N, int M, int dr, int dc, int ds,
                    hipStream_t st);

// Warm-start CNN (cnn.hip).
struct CnnWs {
  uint16_t *wbf;     // bf16 copy of the parameters
  uint16_t *act[5];  // hidden activations [voxel][32] (inference uses act[0..1])
  uint16_t *gz[2];   // gradients at layer outputs
  float *gout, *y, *partial, *lpart;
  size_t bytes;
};
long cnn_param_count();
long cnn_w_offset(int layer);
CnnWs cnn_layout(int S, int N, int M, bool training, char *base);
hipError_t cnn_init(float *params, uint64_t seed, hipStream_t st);
hipError_t cnn_adam(float *p, const float *g, float *m, float *v, int step, float lr, float b1,
                    float b2, float eps, hipStream_t st);
hipError_t cnn_forward(int S, int N, int M, const float *params, const float *x, float *y,
                       const CnnWs &L, bool training, const float *target, float *gout,
                       float *lpart, hipStream_t st);
hipError_t cnn_grad(int S, int N, int M, const float *params, const float *x, const float *target,
                    float *grad, float *loss, const CnnWs &L, hipStream_t st);
hipError_t conv_layer_forward(int S, int N, int M, int cin, int cout, const void *in,
                              const float *x, const uint16_t *wbf, const float *bias, void *out_bf16,
                              float *out_f32, hipStream_t st);
hipError_t conv_layer_backward(int S, int N, int M, const void *act_in, const void *gz,
                               const uint16_t *wbf, const void *mask, void *gin_bf16,
                               float *gin_f32, float *gw, float *partial, hipStream_t st);
size_t conv_layer_partial_bytes(long NV);
hipError_t to_bf16(const float *p, uint16_t *q, long n, hipStream_t st);

}  // namespace sr3d
