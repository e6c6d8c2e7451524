// C ABI of libsr3d: argument checks, workspace layout and the host sequence
// of kernel launches for the Tikhonov closed form (eq. (12)) and TV-ADMM
// (Algorithm 1), with isotropic or anisotropic TV or the l1 norm of Haar
// detail coefficients as the regulariser (the last through the Tikhonov
// x-step).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "sr3d_internal.h"

namespace sr3d {
void release_device_tables();
thread_local std::string g_err;

// ---------------------------------------------------------------------------
// SR3D_PROFILE: HIP events around every launch of the calling thread.
// ---------------------------------------------------------------------------
namespace {
struct ProfState {
  bool active = false;
  int override_stage = -1;
  std::vector<hipEvent_t> pool;
  std::vector<int> stage_of;
  size_t used = 0;
};
thread_local ProfState t_prof;
std::mutex g_prof_mu;
double g_prof_ms[kStCount] = {0};
long g_prof_n[kStCount] = {0};
unsigned g_prof_mask = ~0u;  // stages timed under SR3D_PROFILE
const char *kStageNames[kStCount] = {"fft_r2c_m", "fft_c2c_n", "fft_c2c_s", "fold_solve",
                                     "ifft_c2c_s", "ifft_c2c_n", "ifft_c2r_m", "admm_stencil",
                                     "reduce_test", "solve_s", "stencil_r2c", "wavelet", "setup", "l1_data"};
}  // namespace

void prof_begin(int stage, hipStream_t st) {
  ProfState &p = t_prof;
  if (!p.active) return;
  const int recorded = p.override_stage >= 0 ? p.override_stage : stage;
  if (!((g_prof_mask >> recorded) & 1u)) return;
  while (p.pool.size() < p.used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      p.active = false;
      return;
    }
    p.pool.push_back(e);
  }
  if (p.stage_of.size() < p.pool.size() / 2 + 1) p.stage_of.resize(p.pool.size() / 2 + 1);
  p.stage_of[p.used / 2] = p.override_stage >= 0 ? p.override_stage : stage;
  (void)hipEventRecord(p.pool[p.used++], st);
}

void prof_end(hipStream_t st) {
  ProfState &p = t_prof;
  if (!p.active || (p.used & 1) == 0) return;
  (void)hipEventRecord(p.pool[p.used++], st);
}

// Adds the recorded pairs to the totals; the stream must have been synchronised.
static void prof_flush() {
  ProfState &p = t_prof;
  if (p.used == 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (size_t i = 0; i + 1 < p.used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.pool[i], p.pool[i + 1]) == hipSuccess) {
      g_prof_ms[p.stage_of[i / 2]] += ms;
      g_prof_n[p.stage_of[i / 2]] += 1;
    }
  }
  p.used = 0;
}

struct ProfScope {
  bool on;
  ProfScope(bool enable) : on(enable) {
    if (on) {
      t_prof.active = true;
      t_prof.used = 0;
    }
  }
  ~ProfScope() {
    if (on) {
      prof_flush();
      t_prof.active = false;
      t_prof.override_stage = -1;
    }
  }
};
}  // namespace sr3d

using namespace sr3d;

// Workspace of sr3d_tikhonov_noalloc: a static device array (64 MiB, enough
// for a 128^3 HR volume), held by every device the library runs on until the
// process ends. In host code `scratch` is a host-side stand-in; its device
// address comes from hipGetSymbolAddress, once per device, and only that
// address is handed to kernels.
static __device__ __align__(256) char scratch[SR3D_NOALLOC_SCRATCH_BYTES];

namespace {

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return SR3D_ERR_HIP;
}

#define SR3D_TRY(expr, where)                     \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

bool fold_d_supported(int d) {
  switch (d) {
    case 1: case 2: case 3: case 4: case 6: case 8: case 9: case 12: case 16: case 18: case 24:
    case 27: case 32: case 36: case 48: case 64:
      return true;
    default:
      return false;
  }
}

struct Geometry {
  int S, N, M, Sl, Nl, Ml, Mh, Mlh, D;
  int dr, dc, ds;
  long NH, NL, nspec, nlspec;
  SolveSPlan sp;  // fused x-update plan (TV)
};

// The m and n rate of a volume whose group size is its plan's member bound and
// whose rates are those an instance of the fused x-update is specialised for
// (2 x 2 x 2, 2 x 2 x 4, 4 x 4 x 2), else 0.
static int fixed_rate(const Geometry &g) {
  const int r = g.sp.dm == 32 ? 4 : 2;
  return (g.D == g.sp.dm && g.dr == r && g.dc == r) ? r : 0;
}

int check_geometry(sr3d_dims hr, sr3d_rate rate, const sr3d_dims *psf, Geometry *g) {
  if (hr.m < 1 || hr.n < 1 || hr.s < 1) return fail(SR3D_ERR_INVALID_ARG, "HR dimensions must be >= 1");
  if (rate.dr < 1 || rate.dc < 1 || rate.ds < 1) return fail(SR3D_ERR_INVALID_ARG, "rates must be >= 1");
  if (hr.m % rate.dr || hr.n % rate.dc || hr.s % rate.ds)
    return fail(SR3D_ERR_NOT_DIVISIBLE, "HR dimension not divisible by its decimation rate");
  const long nh = (long)hr.m * hr.n * hr.s;
  if (nh >= (1L << 31)) return fail(SR3D_ERR_UNSUPPORTED_SIZE, "volume has 2^31 or more voxels");
  g->M = hr.m; g->N = hr.n; g->S = hr.s;
  g->dr = rate.dr; g->dc = rate.dc; g->ds = rate.ds;
  g->Ml = hr.m / rate.dr; g->Nl = hr.n / rate.dc; g->Sl = hr.s / rate.ds;
  g->Mh = g->M / 2 + 1; g->Mlh = g->Ml / 2 + 1;
  g->D = rate.dr * rate.dc * rate.ds;
  g->NH = nh;
  g->NL = (long)g->Ml * g->Nl * g->Sl;
  g->nspec = (long)g->S * g->N * g->Mh;
  g->nlspec = (long)g->Sl * g->Nl * g->Mlh;
  const int lens[6] = {g->M, g->N, g->S, g->Ml, g->Nl, g->Sl};
  for (int L : lens)
    if (!fft_len_supported(L))
      return fail(SR3D_ERR_UNSUPPORTED_SIZE,
                  "FFT length " + std::to_string(L) + " not supported (1, 2^a or 3*2^a, <= 1024)");
  if (!fold_d_supported(g->D))
    return fail(SR3D_ERR_UNSUPPORTED_SIZE, "decimation factor d = dr*dc*ds not supported");
  if (psf) {
    if (psf->m < 1 || psf->n < 1 || psf->s < 1) return fail(SR3D_ERR_INVALID_ARG, "PSF dimensions must be >= 1");
    if (psf->m > hr.m || psf->n > hr.n || psf->s > hr.s)
      return fail(SR3D_ERR_PSF_TOO_LARGE, "PSF larger than the HR volume");
  }
  g->sp = solve_s_plan(g->S, g->N, g->M, g->dr, g->dc, g->ds);
  return SR3D_OK;
}

struct Carve {
  char *base;
  size_t off;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct TvWs {
  Ctrl *ctrl;
  void *partS, *partF;
  float *g;
  float2 *lam, *yh, *w, *w2;
  float *nu[2], *theta;
  // fused x-update (when the geometry has a fused plan)
  float2 *lamg, *yg;
  int *tab;
  SolveSArgs *sdesc;
  int nbS, nbF, nbFold, nbFused;
  int nbStile, nbSrow;  // stencil workgroups: tiled kernel, fused stencil + R2C kernel
  bool fused;  // this solve uses the fused x-update (set by the caller)
  bool fsten;  // ... and the stencil with the m-axis R2C fused in
  bool aniso;  // anisotropic TV (SR3D_TV_ANISO)
  bool haar;   // l1 of Haar details (SR3D_REG_HAAR): Tikhonov fold + wavelet kernels
  int levels;  // Haar levels
  int nbSwav;  // workgroups of the wavelet ADMM kernel
  // l1 data term (SR3D_DATA_L1): LR state v, e; DHx, y', dv = v' - v; the LR
  // spectra of DHx, dv and e'; the weights of ||H^T D^T .||; partial sums
  bool l1;
  float *l1v, *l1e, *l1t, *l1yp, *l1dv, *l1w;
  float2 *l1sa, *l1sy, *l1sb, *l1sc;  // spectra of DHx, y', dv, e
  void *partL, *partW;
  int nbL;
  // multi-frame data term (sr3d_tv_admm_mf): the frames' LR spectra and shifts
  int mfF;
  float2 *mfY;
  int mfT[kMaxFrames][3];
};

// Haar levels of SR3D_REG_HAAR (bits 16-19 of the flags; 0 means 1).
int haar_levels(int flags) {
  const int lv = (flags >> 16) & 0xf;
  return lv ? lv : 1;
}

// Workspace of one TV solve. nu[0] is only used when the caller passes no
// state buffer. The fused x-update buffers exist whenever the geometry has a
// fused plan, so the size does not depend on the flags.
size_t tv_layout(const Geometry &g, char *base, TvWs *L) {
  Carve c{base, 0};
  L->nbStile = stencil_plan(g.S, g.N, g.M).blocks;
  L->nbSrow = g.sp.fused && stencil_r2c_fits(g.S, g.N, g.M, g.sp.pitch)
                  ? stencil_r2c_plan(g.S, g.N, g.M).blocks
                  : 0;
  L->nbSwav = wavelet_blocks(g.S, g.N, g.M);
  // the one-pass wavelet kernel has the most workgroups at one level
  const int nb_wf = wavelet_fused_blocks(g.S, g.N, g.M, 1);
  L->nbS = L->nbStile;
  L->fsten = false;
  L->haar = false;
  L->levels = 1;
  FoldArgs fa{};
  fa.Sl = g.Sl; fa.Nl = g.Nl; fa.ml_eff = g.Ml < g.Mh ? g.Ml : g.Mh;
  L->nbFold = fold_blocks(fa);
  L->nbFused = g.sp.fused ? g.sp.units : 0;
  L->nbF = L->nbFold;
  L->fused = false;
  L->ctrl = c.take<Ctrl>(1);
  int nbs_max = L->nbStile > L->nbSrow ? L->nbStile : L->nbSrow;
  nbs_max = nbs_max > L->nbSwav ? nbs_max : L->nbSwav;
  nbs_max = nbs_max > nb_wf ? nbs_max : nb_wf;
  L->partS = c.take<double>((size_t)6 * nbs_max);
  L->partF = c.take<double>((size_t)(L->nbFold > L->nbFused ? L->nbFold : L->nbFused));
  L->g = c.take<float>((size_t)g.M + g.N + g.S);
  L->lam = c.take<float2>(g.nspec);
  L->yh = c.take<float2>(g.nlspec);
  // w holds the fused path's padded spectrum (rows g.sp.pitch apart) too
  L->w = c.take<float2>(g.sp.fused ? (size_t)g.S * g.N * g.sp.pitch : (size_t)g.nspec);
  L->w2 = c.take<float2>(g.nspec);
  L->nu[0] = c.take<float>((size_t)3 * g.NH);
  L->nu[1] = c.take<float>((size_t)3 * g.NH);
  L->theta = c.take<float>(g.NH);
  L->lamg = L->yg = nullptr;
  L->tab = nullptr;
  L->sdesc = nullptr;
  if (g.sp.fused) {
    L->lamg = c.take<float2>((size_t)g.sp.units * g.D * g.sp.gmax);
    L->yg = c.take<float2>((size_t)g.sp.units * g.sp.gmax);
    L->tab = c.take<int>(g.sp.tab.size());
    L->sdesc = c.take<SolveSArgs>(1);
  }
  L->mfF = 0;
  L->mfY = nullptr;
  // l1 data term: LR-sized, about 5 B per HR voxel at d = 8
  L->l1 = false;
  L->nbL = l1_blocks(g.NL);
  L->l1v = c.take<float>(g.NL);
  L->l1t = c.take<float>(g.NL);
  // y', dv and e back to back, and their spectra: one stacked transform
  L->l1yp = c.take<float>((size_t)3 * g.NL);
  L->l1dv = L->l1yp + g.NL;
  L->l1e = L->l1yp + 2 * (size_t)g.NL;
  L->l1w = c.take<float>(g.nlspec);
  L->l1sa = c.take<float2>(g.nlspec);
  L->l1sy = c.take<float2>((size_t)3 * g.nlspec);
  L->l1sb = L->l1sy + g.nlspec;
  L->l1sc = L->l1sy + 2 * (size_t)g.nlspec;
  L->partL = c.take<double>((size_t)5 * L->nbL);
  L->partW = c.take<double>((size_t)2 * l1_blocks(g.nlspec));
  return c.off + 256;
}

void tv_choose_path(const Geometry &g, int flags, TvWs *L) {
  L->fused = g.sp.fused && !(flags & SR3D_UNFUSED);
  L->nbF = L->fused ? L->nbFused : L->nbFold;
  L->fsten = L->fused && L->nbSrow > 0 && !(flags & SR3D_SEPARATE_R2C);
  L->aniso = (flags & SR3D_TV_ANISO) != 0;
  L->haar = (flags & SR3D_REG_HAAR) != 0;
  L->levels = haar_levels(flags);
  L->l1 = (flags & SR3D_DATA_L1) != 0;
  L->nbS = L->fsten ? L->nbSrow : L->nbStile;
  if (L->haar) {
    // The x-step is the Tikhonov solve (A = mu): the fused x-update with
    // tables gm = 1, gn = gs = 0 where the plan applies, else the fold on the
    // natural spectrum. The stencil is replaced by the wavelet kernels.
    L->fsten = false;
    L->nbS = L->levels <= 3 ? wavelet_fused_blocks(g.S, g.N, g.M, L->levels) : L->nbSwav;
  }
}

SolveSArgs make_solve_args(const Geometry &g, const TvWs &L, const sr3d_problem *p) {
  SolveSArgs a{};
  a.W = L.w; a.Lg = L.lamg; a.Yg = L.yg; a.tab = L.tab;
  a.gm = L.g; a.gn = L.g + g.M; a.gs = L.g + g.M + g.N;
  a.S = g.S; a.N = g.N; a.M = g.M; a.Mh = g.Mh; a.Sl = g.Sl; a.Nl = g.Nl; a.Ml = g.Ml;
  a.P = g.sp.pitch;
  a.dr = g.dr; a.dc = g.dc; a.ds = g.ds; a.D = g.D;
  a.NG = g.sp.NG; a.NB = g.sp.NB; a.CB = g.sp.CB; a.gmax = g.sp.gmax; a.units = g.sp.units;
  a.o_p0 = g.sp.o_p0; a.o_cnt = g.sp.o_cnt; a.o_mj = g.sp.o_mj; a.o_nj = g.sp.o_nj;
  a.mu = p->mu;
  a.scale = (float)(1.0 / (double)g.NH);
  a.partial = L.partF; a.ctrl = L.ctrl; a.done = &L.ctrl->done;
  a.a_pos = L.haar ? 1 : 0;
  if (L.l1) {
    // l1 data term: mu -> mu / mu_data; the group means give the LR spectrum
    // of D H x; its own test replaces the data-term partial sums
    a.mu = p->mu / p->mu_data;
    a.partial = nullptr;
    a.dhx = L.l1sa;
  }
  return a;
}

// The frames' LR half spectra of a multi-frame solve, after the single-frame
// workspace.
size_t mf_extra(const Geometry &g, int nframes) {
  return ((size_t)nframes * g.nlspec * sizeof(float2) + 511) & ~(size_t)255;
}

MfArgs make_mf(const Geometry &g, const float2 *lam, const float2 *yf, int nframes,
               const int (*t)[3]) {
  MfArgs a{};
  a.Lam = lam; a.Yf = yf; a.nlspec = g.nlspec; a.F = nframes;
  for (int f = 0; f < nframes; ++f) {
    for (int c = 0; c < 3; ++c) a.t[f][c] = t[f][c];
    // per-member roots of unity, in FP64 (member q = (c dc + b) dr + a)
    for (int q = 0; q < g.D && q < 32; ++q) {
      const int ia = q % g.dr, ib = (q / g.dr) % g.dc, ic = q / (g.dr * g.dc);
      const double ph = 2.0 * M_PI * ((double)(((long)ia * t[f][0]) % g.dr) / g.dr +
                                      (double)(((long)ib * t[f][1]) % g.dc) / g.dc +
                                      (double)(((long)ic * t[f][2]) % g.ds) / g.ds);
      a.r[f][q] = make_float2((float)cos(ph), (float)sin(ph));
    }
  }
  a.twm = twiddles(g.M); a.twn = twiddles(g.N); a.tws = twiddles(g.S);
  a.S = g.S; a.N = g.N; a.M = g.M; a.Mh = g.Mh;
  a.Sl = g.Sl; a.Nl = g.Nl; a.Ml = g.Ml; a.Mlh = g.Mlh;
  a.dr = g.dr; a.dc = g.dc; a.ds = g.ds;
  a.ml_eff = g.Ml < g.Mh ? g.Ml : g.Mh;
  a.scale = (float)(1.0 / (double)g.NH);
  return a;
}

// Argument checks of the multi-frame entry points (host, before any HIP call).
int check_frames(const Geometry &g, int nframes, const float *const *y, const int *shifts) {
  if (nframes < 1 || nframes > kMaxFrames)
    return fail(SR3D_ERR_INVALID_ARG, "nframes must be 1.." + std::to_string(kMaxFrames));
  if (!y || !shifts) return fail(SR3D_ERR_INVALID_ARG, "frames and shifts must be non-NULL");
  for (int f = 0; f < nframes; ++f) {
    if (!y[f]) return fail(SR3D_ERR_INVALID_ARG, "a frame pointer is NULL");
    for (int c = 0; c < 3; ++c)
      if (shifts[3 * f + c] <= -(1 << 20) || shifts[3 * f + c] >= (1 << 20))
        return fail(SR3D_ERR_INVALID_ARG, "shifts must lie in (-2^20, 2^20)");
  }
  if (!fold_mf_supported(g.D, nframes))
    return fail(SR3D_ERR_UNSUPPORTED_SIZE, "multi-frame solves take d in {1, 2, 4, 8, 16, 32}");
  return SR3D_OK;
}

struct TikWs {
  float2 *lam, *yh, *w, *w2;
  float *real;
};

size_t tik_layout(const Geometry &g, char *base, TikWs *L) {
  Carve c{base, 0};
  L->lam = c.take<float2>(g.nspec);
  L->yh = c.take<float2>(g.nlspec);
  L->w = c.take<float2>(g.nspec);
  L->w2 = c.take<float2>(g.nspec);
  L->real = c.take<float>(g.NH);
  return c.off + 256;
}

size_t degrade_layout(const Geometry &g, char *base, TikWs *L) {
  Carve c{base, 0};
  L->lam = c.take<float2>(g.nspec);
  L->w = c.take<float2>(g.nspec);
  L->real = c.take<float>(g.NH);
  L->yh = nullptr;
  L->w2 = nullptr;
  return c.off + 256;
}

FoldArgs make_fold(const Geometry &g) {
  FoldArgs a{};
  a.S = g.S; a.N = g.N; a.M = g.M; a.Mh = g.Mh;
  a.Sl = g.Sl; a.Nl = g.Nl; a.Ml = g.Ml; a.Mlh = g.Mlh;
  a.dr = g.dr; a.dc = g.dc; a.ds = g.ds;
  a.ml_eff = g.Ml < g.Mh ? g.Ml : g.Mh;
  a.scale = (float)(1.0 / (double)g.NH);
  return a;
}

// pinned host copies of the control block, one per calling thread
std::mutex g_host_mu;
std::vector<Ctrl *> g_host_blocks;
thread_local Ctrl *t_host_ctrl = nullptr;

Ctrl *host_ctrl() {
  if (!t_host_ctrl) {
    void *p = nullptr;
    if (hipHostMalloc(&p, sizeof(Ctrl) * 64, hipHostMallocDefault) != hipSuccess) return nullptr;
    t_host_ctrl = reinterpret_cast<Ctrl *>(p);
    std::lock_guard<std::mutex> lk(g_host_mu);
    g_host_blocks.push_back(t_host_ctrl);
  }
  return t_host_ctrl;
}

int check_problem(const sr3d_problem *p, int flags, Geometry *g) {
  if (!p) return fail(SR3D_ERR_INVALID_ARG, "problem is NULL");
  int rc = check_geometry(p->hr, p->rate, &p->psf_dims, g);
  if (rc) return rc;
  if (!p->y || !p->psf || !p->x) return fail(SR3D_ERR_INVALID_ARG, "y, psf and x must be non-NULL");
  if (!(p->lambda_tv > 0.f) || !(p->mu > 0.f) || !isfinite(p->lambda_tv) || !isfinite(p->mu))
    return fail(SR3D_ERR_INVALID_ARG, "lambda_tv and mu must be finite and > 0");
  if (!(p->tol >= 0.f) || !isfinite(p->tol)) return fail(SR3D_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (!isfinite(p->tol_dual)) return fail(SR3D_ERR_INVALID_ARG, "tol_dual must be finite");
  if (p->max_iter < 1) return fail(SR3D_ERR_INVALID_ARG, "max_iter must be >= 1");
  if ((flags & SR3D_RESUME) && !p->state) return fail(SR3D_ERR_INVALID_ARG, "SR3D_RESUME needs problem.state");
  if ((flags & SR3D_WARM_DUAL) && p->x0 && p->x0 == p->x)
    return fail(SR3D_ERR_INVALID_ARG, "SR3D_WARM_DUAL needs x0 distinct from x");
  if (flags & SR3D_REG_HAAR) {
    const int lv = haar_levels(flags), q = 1 << lv;
    if (lv > 8) return fail(SR3D_ERR_INVALID_ARG, "SR3D_HAAR_LEVELS must be at most 8");
    if (g->S % q || g->N % q || g->M % q)
      return fail(SR3D_ERR_INVALID_ARG, "SR3D_REG_HAAR needs every HR dimension a multiple of 2^levels");
    if (flags & (SR3D_TV_ANISO | SR3D_WARM_DUAL))
      return fail(SR3D_ERR_INVALID_ARG, "SR3D_REG_HAAR excludes SR3D_TV_ANISO and SR3D_WARM_DUAL");
  }
  if (flags & SR3D_DATA_L1) {
    if (!(p->mu_data > 0.f) || !isfinite(p->mu_data))
      return fail(SR3D_ERR_INVALID_ARG, "SR3D_DATA_L1 needs mu_data finite and > 0");
    if (flags & (SR3D_REG_HAAR | SR3D_WARM_DUAL | SR3D_RESUME))
      return fail(SR3D_ERR_INVALID_ARG,
                  "SR3D_DATA_L1 excludes SR3D_REG_HAAR, SR3D_WARM_DUAL and SR3D_RESUME");
  }
  if (p->x == p->y || p->x == p->psf) return fail(SR3D_ERR_INVALID_ARG, "x aliases an input");
  return SR3D_OK;
}

// With the fused stencil, every iteration starts from the m-transformed Theta
// in w (the previous stencil writes it), so the setup leaves Theta0 there too.
hipError_t theta0_spectrum(const Geometry &g, const TvWs &L, hipStream_t st) {
  if (!L.fsten) return hipSuccess;
  prof_begin(kStFftR2cM, st);
  const hipError_t e = launch_r2c_m_v(L.theta, L.w, (long)g.S * g.N, g.M,
                                      fft_variant(kFftR2cM, g.M), nullptr, st, L.tab,
                                      L.tab + g.Mh, g.sp.pitch, nullptr);
  prof_end(st);
  return e;
}

// Enqueue setup and initial state (nu in nu0, Theta) for one TV problem.
hipError_t tv_setup(const Geometry &g, const TvWs &L, const sr3d_problem *p, float *nu0, int flags,
                    hipStream_t st) {
  hipError_t e;
  if ((e = ctrl_init(L.ctrl, p->max_iter, p->tol, p->tol_dual, p->mu, p->lambda_tv,
                     1.0 / (double)g.NL, st)))
    return e;
  if ((e = pad_psf(p->psf, p->psf_dims.s, p->psf_dims.n, p->psf_dims.m, L.theta, g.S, g.N, g.M, st))) return e;
  if ((e = fft3d_forward(L.theta, L.lam, g.S, g.N, g.M, nullptr, st))) return e;
  if ((e = fft3d_forward(p->y, L.yh, g.Sl, g.Nl, g.Ml, nullptr, st))) return e;
  if ((e = diff_tables(L.g, g.S, g.N, g.M, st))) return e;
  if (L.fused) {
    // Plan tables, the kernel's argument block, and Lambda / Y in unit order.
    const SolveSArgs sa = make_solve_args(g, L, p);
    if ((e = hipMemcpyAsync(L.tab, g.sp.tab.data(), sizeof(int) * g.sp.tab.size(),
                            hipMemcpyHostToDevice, st)))
      return e;
    if ((e = hipMemcpyAsync(L.sdesc, &sa, sizeof sa, hipMemcpyHostToDevice, st))) return e;
    if ((e = solve_s_gather(sa, L.lam, L.yh, g.Mlh, st))) return e;
    std::vector<float> gtab;
    if (L.haar) {
      // A = mu * (gm + gn + gs) = mu at every member
      gtab.assign((size_t)g.M + g.N + g.S, 0.f);
      for (int i = 0; i < g.M; ++i) gtab[i] = 1.f;
      if ((e = hipMemcpyAsync(L.g, gtab.data(), sizeof(float) * gtab.size(), hipMemcpyHostToDevice,
                              st)))
        return e;
    }
    if ((e = hipStreamSynchronize(st))) return e;  // the host images above are locals
  }
  const float thr = p->lambda_tv / p->mu;
  if (L.haar) {
    // nu0 = W x0 (d = 0), or the given state; then xbar = W^T (u - d).
    if (L.levels <= 3) {
      const bool resume = (flags & SR3D_RESUME) != 0;
      return wavelet_fused(p->x0, resume ? nu0 : nullptr, resume ? nullptr : nu0, L.theta, g.S,
                           g.N, g.M, L.levels, thr, resume ? 2 : 1, nullptr, false, nullptr, st);
    }
    if (flags & SR3D_RESUME) {
      if ((e = wavelet_admm(L.theta, nu0, nullptr, g.S, g.N, g.M, L.levels, thr, 2, nullptr, false,
                            nullptr, st)))
        return e;
    } else {
      if (p->x0) e = haar3(p->x0, L.theta, g.S, g.N, g.M, L.levels, false, nullptr, st);
      else e = fill_zero(L.theta, (size_t)g.NH, st);
      if (e) return e;
      if ((e = wavelet_admm(L.theta, nullptr, nu0, g.S, g.N, g.M, L.levels, thr, 1, nullptr, false,
                            nullptr, st)))
        return e;
    }
    return haar3(nullptr, L.theta, g.S, g.N, g.M, L.levels, true, nullptr, st);
  }
  if (flags & SR3D_RESUME) {
    if ((e = theta_from_nu(nu0, L.theta, g.S, g.N, g.M, thr, L.aniso, st))) return e;
    return theta0_spectrum(g, L, st);
  }
  const float *xinit = p->x0;
  if (p->x0 && (flags & SR3D_WARM_DUAL)) {
    // nu0 = L (x0 + phi): u0 = shrink(nu0), d0 = nu0 - u0 start from the
    // minimum-norm dual that makes x0 stationary for the x-update.
    if ((e = fft3d_forward(p->x0, L.w, g.S, g.N, g.M, nullptr, st))) return e;
    FoldArgs fa = make_fold(g);
    fa.W = L.w; fa.Lam = L.lam; fa.Yh = L.yh; fa.X = L.w2;
    fa.gm = L.g; fa.gn = L.g + g.M; fa.gs = L.g + g.M + g.N;
    fa.coefA = p->mu;
    if ((e = dual_init_spectrum(fa, st))) return e;
    if ((e = fft3d_inverse(L.w2, p->x, g.S, g.N, g.M, 1.0f, nullptr, st))) return e;
    if ((e = add_to(p->x, p->x0, (size_t)g.NH, st))) return e;
    xinit = p->x;
  }
  AdmmStencilArgs sa{};
  sa.x = xinit; sa.nu_in = nullptr; sa.nu_out = nu0; sa.theta = L.theta;
  sa.S = g.S; sa.N = g.N; sa.M = g.M; sa.thr = thr; sa.part = nullptr; sa.done = nullptr;
  sa.aniso = L.aniso ? 1 : 0;
  if ((e = admm_stencil(sa, false, false, st))) return e;
  return theta0_spectrum(g, L, st);
}

// One iteration of the wavelet form: x-step by the Tikhonov fold (A = mu,
// xbar in theta), then W, steps 5b/5c and W^T back into theta. On the fused
// path the stopping test is carried by the next iteration's R2C as for TV.
hipError_t wavelet_iteration(const Geometry &g, const TvWs &L, const sr3d_problem *p,
                             float *const nu[2], int k, bool fp64, hipStream_t st, bool merged,
                             bool last) {
  const int *done = &L.ctrl->done;
  hipError_t e;
  const bool carry = L.fused && g.M > 1;
  if (L.fused) {
    const int *kofp = L.tab, *posk = L.tab + g.Mh;
    const RedArgs red{L.ctrl, L.partS, L.nbS, L.partF, L.nbF, fp64 ? 1 : 0};
    if ((e = fft2d_mn_forward(L.theta, L.w, g.S, g.N, g.M, kofp, posk, g.sp.pitch, done, st,
                              carry && merged ? &red : nullptr)))
      return e;
    prof_begin(kStSolveS, st);
    e = solve_s(g.S, g.sp.dm, g.D, fixed_rate(g), L.sdesc, nullptr, g.sp.units, fp64, st);
    prof_end(st);
    if (e) return e;
    if ((e = fft2d_mn_inverse(L.w, p->x, g.S, g.N, g.M, 1.0f, kofp, posk, g.sp.pitch, done, st)))
      return e;
  } else {
    if ((e = fft3d_forward(L.theta, L.w, g.S, g.N, g.M, done, st))) return e;
    FoldArgs fa = make_fold(g);
    fa.W = L.w; fa.Lam = L.lam; fa.Yh = L.yh; fa.X = L.w2;
    fa.cw = p->mu; fa.coefA = p->mu; fa.tv = 0;
    fa.partial = L.partF; fa.ctrl = L.ctrl; fa.done = done;
    if ((e = fold_solve(fa, fp64, st))) return e;
    if ((e = fft3d_inverse(L.w2, p->x, g.S, g.N, g.M, 1.0f, done, st))) return e;
  }
  prof_begin(kStWavelet, st);
  const float thr = p->lambda_tv / p->mu;
  if (L.levels <= 3) {
    e = wavelet_fused(p->x, nu[(k - 1) & 1], nu[k & 1], L.theta, g.S, g.N, g.M, L.levels, thr, 0,
                      L.partS, fp64, done, st);
  } else {
    e = haar3(p->x, L.theta, g.S, g.N, g.M, L.levels, false, done, st);
    if (!e)
      e = wavelet_admm(L.theta, nu[(k - 1) & 1], nu[k & 1], g.S, g.N, g.M, L.levels, thr, 0,
                       L.partS, fp64, done, st);
    if (!e) e = haar3(nullptr, L.theta, g.S, g.N, g.M, L.levels, true, done, st);
  }
  prof_end(st);
  if (e) return e;
  if (carry && !last) return hipSuccess;  // reduced by the next iteration's first launch
  return reduce_and_test(L.ctrl, L.partS, L.nbS, L.partF, L.nbF, fp64, st);
}

// l1 data term, initialisation: steps 5b'/5c' applied to x0 with zero
// duals (a = D H x0 - y, v = soft(a, 1/mu_data), e = a - v), y' = y + v - e
// and its LR spectrum for the first x-step; the weights of ||H^T D^T .||.
// `tmp` is an HR scratch volume (the state buffer the first iteration writes).
hipError_t l1_setup(const Geometry &g, const TvWs &L, const sr3d_problem *p, float *tmp,
                    hipStream_t st) {
  hipError_t e;
  if ((e = l1_weights(L.lam, L.l1w, g.S, g.N, g.M, g.dr, g.dc, g.ds, st))) return e;
  const float *t = nullptr;  // D H x0 (x0 = 0: none)
  if (p->x0) {
    if ((e = fft3d_forward(p->x0, L.w2, g.S, g.N, g.M, nullptr, st))) return e;
    if ((e = spectrum_mul(L.w2, L.lam, (size_t)g.nspec, (float)(1.0 / (double)g.NH), st))) return e;
    if ((e = fft3d_inverse(L.w2, tmp, g.S, g.N, g.M, 1.0f, nullptr, st))) return e;
    if ((e = decimate(tmp, L.l1t, g.S, g.N, g.M, g.dr, g.dc, g.ds, st))) return e;
    t = L.l1t;
  }
  if ((e = l1_update(t, p->y, L.l1v, L.l1e, L.l1yp, nullptr, g.NL, 1.0f / p->mu_data, true, nullptr,
                     false, nullptr, st)))
    return e;
  return fft3d_forward(L.l1yp, L.l1sy, g.Sl, g.Nl, g.Ml, nullptr, st);
}

// One iteration with the l1 data term: the x-step of Algorithm 1 with
// y -> y' (its LR spectrum in yh) and mu -> mu / mu_data, through the fused
// x-update where the plan applies (else the fold on the natural spectrum),
// either of which also leaves the LR spectrum of D H x; steps 5b/5c
// (threshold lam / mu); then on the LR grid D H x, steps 5b'/5c', the
// spectrum of the next y', the data split's dual norms, and the stopping test
// over both splits.
hipError_t l1_iteration(const Geometry &g, const TvWs &L, const sr3d_problem *p, float *const nu[2],
                        int k, bool fp64, hipStream_t st) {
  const int *done = &L.ctrl->done;
  hipError_t e;
  if (L.fused) {
    // The fused x-update, with y' (new every iteration) gathered into unit
    // order; its group means leave the LR spectrum of D H x.
    const int *kofp = L.tab, *posk = L.tab + g.Mh;
    if ((e = solve_s_gather_y(make_solve_args(g, L, p), L.l1sy, g.Mlh, st))) return e;
    if (L.fsten)
      e = fft_n_forward(L.w, g.S, g.N, g.M, g.sp.pitch, done, st, nullptr);
    else
      e = fft2d_mn_forward(L.theta, L.w, g.S, g.N, g.M, kofp, posk, g.sp.pitch, done, st, nullptr);
    if (e) return e;
    prof_begin(kStSolveS, st);
    e = solve_s(g.S, g.sp.dm, g.D, fixed_rate(g), L.sdesc, nullptr, g.sp.units, fp64, st);
    prof_end(st);
    if (e) return e;
    if ((e = fft2d_mn_inverse(L.w, p->x, g.S, g.N, g.M, 1.0f, kofp, posk, g.sp.pitch, done, st)))
      return e;
  } else {
    if ((e = fft3d_forward(L.theta, L.w, g.S, g.N, g.M, done, st))) return e;
    const float mur = p->mu / p->mu_data;
    FoldArgs fa = make_fold(g);
    fa.W = L.w; fa.Lam = L.lam; fa.Yh = L.l1sy; fa.X = L.w2;
    fa.gm = L.g; fa.gn = L.g + g.M; fa.gs = L.g + g.M + g.N;
    fa.cw = mur; fa.coefA = mur; fa.tv = 1;
    fa.partial = nullptr; fa.ctrl = L.ctrl; fa.done = done; fa.dhx = L.l1sa;
    if ((e = fold_solve(fa, fp64, st))) return e;
    if ((e = fft3d_inverse(L.w2, p->x, g.S, g.N, g.M, 1.0f, done, st))) return e;
  }
  AdmmStencilArgs sa{};
  sa.x = p->x; sa.nu_in = nu[(k - 1) & 1]; sa.nu_out = nu[k & 1]; sa.theta = L.theta;
  sa.S = g.S; sa.N = g.N; sa.M = g.M; sa.thr = p->lambda_tv / p->mu;
  sa.part = L.partS; sa.done = done; sa.aniso = L.aniso ? 1 : 0;
  if (L.fsten)
    e = admm_stencil_r2c(sa, L.w, L.tab, g.sp.pitch, fp64, st);
  else
    e = admm_stencil(sa, true, fp64, st);
  if (e) return e;
  const int saved = t_prof.override_stage;
  t_prof.override_stage = kStL1Data;
  e = fft3d_inverse(L.l1sa, L.l1t, g.Sl, g.Nl, g.Ml, (float)(1.0 / (double)g.NL), done, st);
  if (!e) {
    prof_begin(kStL1Data, st);
    e = l1_update(L.l1t, p->y, L.l1v, L.l1e, L.l1yp, L.l1dv, g.NL, 1.0f / p->mu_data, false,
                  L.partL, fp64, done, st);
    prof_end(st);
  }
  if (!e) e = fft3d_forward_stack(L.l1yp, L.l1sy, 3, g.Sl, g.Nl, g.Ml, done, st);  // y', dv, e
  if (!e) {
    prof_begin(kStL1Data, st);
    e = l1_wnorm(L.l1sb, L.l1sc, L.l1w, g.nlspec, L.partW, fp64, done, st);
    prof_end(st);
  }
  t_prof.override_stage = saved;
  if (e) return e;
  return l1_reduce_test(L.ctrl, L.partS, L.nbS, L.partL, L.nbL, L.partW, l1_blocks(g.nlspec), fp64,
                        st);
}

// Enqueue iteration k (1-based): reads nu[(k-1)%2], writes nu[k%2]. The
// stopping test of an iteration runs in an extra workgroup of the next
// iteration's first launch (fused path, not the first iteration of an
// enqueued chunk: `merged`), or in its own launch at the end of a chunk
// (`last`), so the host sees complete statistics after every chunk.
hipError_t tv_iteration(const Geometry &g, const TvWs &L, const sr3d_problem *p, float *const nu[2],
                        int k, bool fp64, hipStream_t st, bool merged, bool last) {
  if (L.haar) return wavelet_iteration(g, L, p, nu, k, fp64, st, merged, last);
  if (L.l1) return l1_iteration(g, L, p, nu, k, fp64, st);
  const int *done = &L.ctrl->done;
  hipError_t e;
  // The iteration's first launch can carry the previous reduction: the R2C
  // (m = 1 uses a plain copy kernel), or with the fused stencil, whose m pass
  // is already done, the n pass (none for n = 1).
  const bool carry = L.fsten ? g.N > 1 : L.fused && g.M > 1;
  if (L.fused) {
    const int *kofp = L.tab, *posk = L.tab + g.Mh;
    const RedArgs red{L.ctrl, L.partS, L.nbS, L.partF, L.nbF, fp64 ? 1 : 0};
    if (L.fsten)
      e = fft_n_forward(L.w, g.S, g.N, g.M, g.sp.pitch, done, st, carry && merged ? &red : nullptr);
    else
      e = fft2d_mn_forward(L.theta, L.w, g.S, g.N, g.M, kofp, posk, g.sp.pitch, done, st,
                           carry && merged ? &red : nullptr);
    if (e) return e;
    prof_begin(kStSolveS, st);
    e = solve_s(g.S, g.sp.dm, g.D, fixed_rate(g), L.sdesc, nullptr, g.sp.units, fp64, st);
    prof_end(st);
    if (e) return e;
    if ((e = fft2d_mn_inverse(L.w, p->x, g.S, g.N, g.M, 1.0f, kofp, posk, g.sp.pitch, done, st)))
      return e;
  } else {
    if ((e = fft3d_forward(L.theta, L.w, g.S, g.N, g.M, done, st))) return e;
    if (L.mfF) {
      MfArgs ma = make_mf(g, L.lam, L.mfY, L.mfF, L.mfT);
      ma.W = L.w; ma.X = L.w2;
      ma.gm = L.g; ma.gn = L.g + g.M; ma.gs = L.g + g.M + g.N;
      ma.cw = p->mu; ma.coefA = p->mu; ma.tv = 1;
      ma.partial = L.partF; ma.ctrl = L.ctrl; ma.done = done;
      if ((e = fold_solve_mf(ma, fp64, st))) return e;
    } else {
      FoldArgs fa = make_fold(g);
      fa.W = L.w; fa.Lam = L.lam; fa.Yh = L.yh; fa.X = L.w2;
      fa.gm = L.g; fa.gn = L.g + g.M; fa.gs = L.g + g.M + g.N;
      fa.cw = p->mu; fa.coefA = p->mu; fa.tv = 1;
      fa.partial = L.partF; fa.ctrl = L.ctrl; fa.done = done;
      if ((e = fold_solve(fa, fp64, st))) return e;
    }
    if ((e = fft3d_inverse(L.w2, p->x, g.S, g.N, g.M, 1.0f, done, st))) return e;
  }
  AdmmStencilArgs sa{};
  sa.x = p->x; sa.nu_in = nu[(k - 1) & 1]; sa.nu_out = nu[k & 1]; sa.theta = L.theta;
  sa.S = g.S; sa.N = g.N; sa.M = g.M; sa.thr = p->lambda_tv / p->mu;
  sa.part = L.partS; sa.done = done; sa.aniso = L.aniso ? 1 : 0;
  if (L.fsten)
    e = admm_stencil_r2c(sa, L.w, L.tab, g.sp.pitch, fp64, st);
  else
    e = admm_stencil(sa, true, fp64, st);
  if (e) return e;
  if (carry && !last) return hipSuccess;  // reduced by the next iteration's first launch
  return reduce_and_test(L.ctrl, L.partS, L.nbS, L.partF, L.nbF, fp64, st);
}

int check_interval(int flags) {
  const int k = (flags >> 8) & 0xff;
  return k > 0 ? k : 8;
}

// nframes > 0: the multi-frame data term over frames[0..nframes-1] with HR
// shifts `shifts` ([nframes][3], host); p->y is not read then.
int run_tv(const sr3d_problem *p, int flags, sr3d_stats *stats, void *ws, size_t ws_bytes,
           hipStream_t st, int nframes = 0, const float *const *frames = nullptr,
           const int *shifts = nullptr) {
  Geometry g;
  int rc = check_problem(p, flags, &g);
  if (rc) return rc;
  if (nframes > 0) {
    if ((rc = check_frames(g, nframes, frames, shifts))) return rc;
    if (flags & (SR3D_REG_HAAR | SR3D_WARM_DUAL | SR3D_DATA_L1))
      return fail(SR3D_ERR_INVALID_ARG,
                  "multi-frame solves exclude SR3D_REG_HAAR, SR3D_WARM_DUAL and SR3D_DATA_L1");
  }
  TvWs L;
  const size_t base_need = tv_layout(g, nullptr, &L);
  const size_t need = base_need + (nframes > 0 ? mf_extra(g, nframes) : 0);
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  tv_layout(g, reinterpret_cast<char *>(ws), &L);
  tv_choose_path(g, flags, &L);
  if (nframes > 0) {
    // the multi-frame fold runs on the natural spectrum
    L.mfF = nframes;
    L.mfY = reinterpret_cast<float2 *>(reinterpret_cast<char *>(ws) + base_need);
    for (int f = 0; f < nframes; ++f)
      for (int c = 0; c < 3; ++c) L.mfT[f][c] = shifts[3 * f + c];
    L.fused = false;
    L.fsten = false;
    L.nbF = L.nbFold;
    L.nbS = L.nbStile;
  }
  Ctrl *hc = host_ctrl();
  if (!hc) return fail(SR3D_ERR_HIP, "hipHostMalloc failed");
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  const bool fp64 = (flags & SR3D_FP64_REDUCE) != 0;
  float *nu[2] = {p->state ? p->state : L.nu[0], L.nu[1]};
  ProfScope prof((flags & SR3D_PROFILE) && !(flags & SR3D_USE_GRAPH));
  t_prof.override_stage = prof.on ? kStSetup : -1;
  SR3D_TRY(tv_setup(g, L, p, nu[0], flags, st), "tv setup");
  if (L.l1) SR3D_TRY(l1_setup(g, L, p, nu[1], st), "l1 data setup");
  for (int f = 0; f < L.mfF; ++f)
    SR3D_TRY(fft3d_forward(frames[f], L.mfY + (size_t)f * g.nlspec, g.Sl, g.Nl, g.Ml, nullptr, st),
             "frame spectra");
  t_prof.override_stage = -1;
  int K = check_interval(flags);
  if (flags & SR3D_USE_GRAPH) {
    // Capture K iterations (K even, so the two state buffers alternate the
    // same way in every replay) on a private stream; replay until done.
    K += K & 1;
    hipStream_t cs;
    SR3D_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream create");
    hipEvent_t ev;
    SR3D_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int i = 1; e == hipSuccess && i <= K; ++i)
      e = tv_iteration(g, L, p, nu, i, fp64, cs, i > 1, i == K);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    for (int it = 0; e == hipSuccess && it < p->max_iter; it += K) {
      e = hipGraphLaunch(exec, cs);
      if (e == hipSuccess) e = hipMemcpyAsync(hc, L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, cs);
      if (e == hipSuccess) e = hipStreamSynchronize(cs);
      if (e == hipSuccess && hc->done) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipEventRecord(ev, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    (void)hipStreamSynchronize(cs);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "graph replay");
  } else {
    for (int it = 0; it < p->max_iter;) {
      const int n = (p->max_iter - it) < K ? (p->max_iter - it) : K;
      for (int i = 1; i <= n; ++i)
        SR3D_TRY(tv_iteration(g, L, p, nu, it + i, fp64, st, i > 1, i == n), "tv iteration");
      it += n;
      SR3D_TRY(hipMemcpyAsync(hc, L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "ctrl copy");
      SR3D_TRY(hipStreamSynchronize(st), "stream sync");
      if (prof.on) prof_flush();
      if (hc->done) break;
    }
  }
  // The latest state is in nu[iter % 2]; hand it back in the caller's buffer.
  if (p->state && (hc->iter & 1)) {
    SR3D_TRY(hipMemcpyAsync(p->state, nu[1], sizeof(float) * 3 * (size_t)g.NH,
                            hipMemcpyDeviceToDevice, st), "state copy");
    SR3D_TRY(hipStreamSynchronize(st), "stream sync");
  }
  if (stats) {
    stats->iters = hc->iter;
    stats->converged = hc->converged;
    stats->primal_rel = hc->primal_rel;
    stats->dual_rel = hc->dual_rel;
    stats->objective = hc->objective;
  }
  if (hc->status) {
    return fail(hc->status, hc->status == SR3D_ERR_SINGULAR ? "Lambda(0) = 0: TV x-update singular"
                                                            : "non-finite residual");
  }
  return SR3D_OK;
}


// ---------------------------------------------------------------------------
// Batched solve: many volumes, every stage launched once per FFT-length (or
// decimation-factor) class over a work list of (volume, tile) items.
// ---------------------------------------------------------------------------

struct BatchPlan {
  struct Group {
    int kind;     // 0..5 FFT kinds, 6 fold, 7 stencil, 8 fused x-update,
                  // 9 stencil with the m-axis R2C fused in
    int key;      // FFT length / decimation factor
    int variant;  // FFT tile variant
    std::vector<int2> items;
    size_t off;   // byte offset of the items in the device header
  };
  std::vector<Group> groups;
};

// Header bytes for `count` volumes and the given items.
struct BatchHeader {
  RowDesc *r2c, *c2r;
  StridedDesc *fn, *in_, *fs, *is;
  FoldArgs *fold;
  SolveSArgs *solve;
  BatchStencilDesc *sten;
  ReduceDesc *red;
  int *active;
  int2 *items;
  size_t bytes;
};

size_t batch_header(int count, size_t nitems, char *base, BatchHeader *H) {
  Carve c{base, 0};
  H->r2c = c.take<RowDesc>(count);
  H->c2r = c.take<RowDesc>(count);
  H->fn = c.take<StridedDesc>(count);
  H->in_ = c.take<StridedDesc>(count);
  H->fs = c.take<StridedDesc>(count);
  H->is = c.take<StridedDesc>(count);
  H->fold = c.take<FoldArgs>(count);
  H->solve = c.take<SolveSArgs>(count);
  H->sten = c.take<BatchStencilDesc>(count);
  H->red = c.take<ReduceDesc>(count);
  H->active = c.take<int>(64);
  H->items = c.take<int2>(nitems);
  H->bytes = c.off + 256;
  return H->bytes;
}

// Items of every (stage, class) group for volumes with geometries g; fused[v]
// selects the fused x-update (kind 8, key S, variant = member bound) for
// volume v instead of the s-FFTs and the fold.
size_t batch_items(const std::vector<Geometry> &g, const std::vector<char> &fused,
                   const std::vector<char> &fsten, BatchPlan *plan) {
  plan->groups.clear();
  auto group = [&](int kind, int key, int variant) -> BatchPlan::Group & {
    for (auto &x : plan->groups)
      if (x.kind == kind && x.key == key && x.variant == variant) return x;
    plan->groups.push_back(BatchPlan::Group{kind, key, variant, {}, 0});
    return plan->groups.back();
  };
  const int n = (int)g.size();
  for (int kind = 0; kind < kFftKinds; ++kind) {
    for (int v = 0; v < n; ++v) {
      const Geometry &G = g[v];
      const long Mh = G.Mh;
      int len, tiles;
      if (kind == kFftR2cM || kind == kFftC2rM) {
        len = G.M;
        if (len == 1) continue;  // copy kernels, launched per volume
        if (kind == kFftR2cM && fsten[v]) continue;  // done by the fused stencil
        tiles = row_tiles(len, fft_variant(kind, len), (long)G.S * G.N);
      } else if (kind == kFftFwdN || kind == kFftInvN) {
        len = G.N;
        if (len == 1) continue;
        tiles = strided_tiles(len, fft_variant(kind, len), (long)G.S * (fused[v] ? G.sp.pitch : Mh));
      } else {
        len = G.S;
        if (len == 1 || fused[v]) continue;
        tiles = strided_tiles(len, fft_variant(kind, len), (long)G.N * Mh);
      }
      auto &gr = group(kind, len, fft_variant(kind, len));
      for (int t = 0; t < tiles; ++t) gr.items.push_back(make_int2(v, t));
    }
  }
  for (int v = 0; v < n; ++v) {
    if (fused[v]) {
      // variant: 4 x member bound, +1 for the instance with the group size
      // fixed, +2 for the instance with the m and n rates fixed as well
      auto &gr = group(8, g[v].S,
                       4 * g[v].sp.dm + (g[v].D == g[v].sp.dm ? 1 : 0) + (fixed_rate(g[v]) ? 2 : 0));
      for (int t = 0; t < g[v].sp.units; ++t) gr.items.push_back(make_int2(v, t));
      continue;
    }
    FoldArgs fa = make_fold(g[v]);
    auto &gr = group(6, g[v].D, 0);
    const int nb = fold_blocks(fa);
    for (int t = 0; t < nb; ++t) gr.items.push_back(make_int2(v, t));
  }
  for (int v = 0; v < n; ++v) {
    if (fsten[v]) {
      auto &gr = group(9, g[v].M, 0);
      const int nb = stencil_r2c_plan(g[v].S, g[v].N, g[v].M).blocks;
      for (int t = 0; t < nb; ++t) gr.items.push_back(make_int2(v, t));
    } else {
      auto &gr = group(7, 0, 0);
      const int nb = stencil_plan(g[v].S, g[v].N, g[v].M).blocks;
      for (int t = 0; t < nb; ++t) gr.items.push_back(make_int2(v, t));
    }
  }
  size_t total = 0;
  for (auto &x : plan->groups) total += x.items.size();
  return total;
}

// Workspace of a batch: header (descriptors and items) then one TV
// workspace per volume. The header holds the larger of the fused and the
// unfused item lists, so the size does not depend on the flags; `plan`
// receives the items for `unfused`.
// The header is sized for the largest item list any flags can choose
// (unfused; fused with the separate stencil and R2C; fused with the fused
// stencil), so the workspace size does not depend on the flags; `plan` is the
// one `flags` choose.
size_t batch_workspace(const sr3d_problem *p, int count, int flags, std::vector<Geometry> *gs,
                       std::vector<size_t> *offs, BatchPlan *plan, size_t *header) {
  gs->resize(count);
  for (int i = 0; i < count; ++i)
    if (check_geometry(p[i].hr, p[i].rate, &p[i].psf_dims, &(*gs)[i])) return 0;
  std::vector<char> fz(count), fs(count), none(count, 0);
  for (int i = 0; i < count; ++i) {
    fz[i] = (*gs)[i].sp.fused ? 1 : 0;
    const Geometry &gi = (*gs)[i];
    fs[i] = fz[i] && stencil_r2c_fits(gi.S, gi.N, gi.M, gi.sp.pitch) ? 1 : 0;
  }
  const bool unfused = (flags & SR3D_UNFUSED) != 0, separate = (flags & SR3D_SEPARATE_R2C) != 0;
  BatchPlan other;
  const size_t n_unf = batch_items(*gs, none, none, unfused ? plan : &other);
  const size_t n_sep = batch_items(*gs, fz, none, !unfused && separate ? plan : &other);
  const size_t n_fst = batch_items(*gs, fz, fs, !unfused && !separate ? plan : &other);
  size_t nitems = n_unf > n_sep ? n_unf : n_sep;
  nitems = nitems > n_fst ? nitems : n_fst;
  BatchHeader H;
  *header = batch_header(count, nitems, nullptr, &H);
  size_t off = (*header + 255) & ~(size_t)255;
  offs->resize(count);
  for (int i = 0; i < count; ++i) {
    TvWs L;
    (*offs)[i] = off;
    off += (tv_layout((*gs)[i], nullptr, &L) + 255) & ~(size_t)255;
  }
  return off;
}

hipError_t batch_iteration(const BatchPlan &plan, const BatchHeader &H,
                           const std::vector<Geometry> &g, const std::vector<TvWs> &Ls,
                           const sr3d_problem *p, int k, bool fp64, hipStream_t st) {
  const int n = (int)g.size();
  hipError_t e = hipSuccess;
  auto items_of = [&](const BatchPlan::Group &gr) {
    return reinterpret_cast<const int2 *>(reinterpret_cast<const char *>(H.items) + gr.off);
  };
  auto run_fft = [&](int kind, int stage) -> hipError_t {
    for (auto &gr : plan.groups) {
      if (gr.kind != kind) continue;
      prof_begin(stage, st);
      hipError_t r;
      const int ni = (int)gr.items.size();
      switch (kind) {
        case kFftR2cM: r = launch_rows_batch(gr.key, false, gr.variant, H.r2c, items_of(gr), ni, st); break;
        case kFftC2rM: r = launch_rows_batch(gr.key, true, gr.variant, H.c2r, items_of(gr), ni, st); break;
        case kFftFwdN: r = launch_strided_batch(gr.key, false, gr.variant, H.fn, items_of(gr), ni, st); break;
        case kFftInvN: r = launch_strided_batch(gr.key, true, gr.variant, H.in_, items_of(gr), ni, st); break;
        case kFftFwdS: r = launch_strided_batch(gr.key, false, gr.variant, H.fs, items_of(gr), ni, st); break;
        default: r = launch_strided_batch(gr.key, true, gr.variant, H.is, items_of(gr), ni, st); break;
      }
      prof_end(st);
      if (r != hipSuccess) return r;
    }
    // volumes with m = 1 use the per-volume copy kernels
    if (kind == kFftR2cM || kind == kFftC2rM)
      for (int v = 0; v < n; ++v) {
        if (g[v].M != 1) continue;
        const Geometry &G = g[v];
        hipError_t r = (kind == kFftR2cM)
                           ? launch_r2c_m_v(Ls[v].theta, Ls[v].w, (long)G.S * G.N, 1, 0, &Ls[v].ctrl->done, st)
                           : launch_c2r_m_v(Ls[v].fused ? Ls[v].w : Ls[v].w2, p[v].x, (long)G.S * G.N, 1,
                                            1.0f, 0, &Ls[v].ctrl->done, st);
        if (r != hipSuccess) return r;
      }
    return hipSuccess;
  };
  if ((e = run_fft(kFftR2cM, kStFftR2cM))) return e;
  if ((e = run_fft(kFftFwdN, kStFftN))) return e;
  if ((e = run_fft(kFftFwdS, kStFftS))) return e;
  for (auto &gr : plan.groups) {
    if (gr.kind != 8) continue;
    prof_begin(kStSolveS, st);
    const int dm = gr.variant / 4;
    e = solve_s(gr.key, dm, (gr.variant & 1) ? dm : -1, (gr.variant & 2) ? (dm == 32 ? 4 : 2) : 0,
                H.solve, items_of(gr), (int)gr.items.size(), fp64, st);
    prof_end(st);
    if (e) return e;
  }
  for (auto &gr : plan.groups) {
    if (gr.kind != 6) continue;
    prof_begin(kStFold, st);
    e = fold_solve_batch(gr.key, H.fold, items_of(gr), (int)gr.items.size(), fp64, st);
    prof_end(st);
    if (e) return e;
  }
  if ((e = run_fft(kFftInvS, kStIfftS))) return e;
  if ((e = run_fft(kFftInvN, kStIfftN))) return e;
  if ((e = run_fft(kFftC2rM, kStIfftC2rM))) return e;
  for (auto &gr : plan.groups) {
    if (gr.kind != 7) continue;
    prof_begin(kStStencil, st);
    // the flags, and so the regulariser, are the same for every volume
    e = admm_stencil_batch(H.sten, items_of(gr), (int)gr.items.size(), k, fp64, Ls[0].aniso, st);
    prof_end(st);
    if (e) return e;
  }
  for (auto &gr : plan.groups) {
    if (gr.kind != 9) continue;
    prof_begin(kStStencilR2c, st);
    e = admm_stencil_r2c_batch(gr.key, H.sten, items_of(gr), (int)gr.items.size(), k, fp64,
                               Ls[0].aniso, st);
    prof_end(st);
    if (e) return e;
  }
  prof_begin(kStReduce, st);
  e = reduce_and_test_batch(H.red, n, H.active, fp64, st);
  prof_end(st);
  return e;
}

int run_batch(const sr3d_problem *p, int count, int flags, sr3d_stats *stats, void *ws,
              size_t ws_bytes, hipStream_t st) {
  if (!p || count < 1) return fail(SR3D_ERR_INVALID_ARG, "no problems");
  if (flags & (SR3D_REG_HAAR | SR3D_DATA_L1))
    return fail(SR3D_ERR_INVALID_ARG, "SR3D_REG_HAAR and SR3D_DATA_L1 are not supported by sr3d_batch");
  Geometry g0;
  for (int i = 0; i < count; ++i) {
    int rc = check_problem(&p[i], flags, &g0);
    if (rc) return rc;
  }
  std::vector<Geometry> g;
  std::vector<size_t> offs;
  BatchPlan plan;
  size_t hdr = 0;
  const size_t need = batch_workspace(p, count, flags, &g, &offs, &plan, &hdr);
  if (!need) return fail(SR3D_ERR_INVALID_ARG, "invalid geometry");
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  char *base = reinterpret_cast<char *>(ws);
  BatchHeader H;
  size_t nitems = 0;
  for (auto &gr : plan.groups) nitems += gr.items.size();
  batch_header(count, nitems, base, &H);
  std::vector<TvWs> Ls(count);
  for (int i = 0; i < count; ++i) {
    tv_layout(g[i], base + offs[i], &Ls[i]);
    tv_choose_path(g[i], flags, &Ls[i]);
  }
  Ctrl *hc = host_ctrl();
  if (!hc) return fail(SR3D_ERR_HIP, "hipHostMalloc failed");
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  const bool fp64 = (flags & SR3D_FP64_REDUCE) != 0;
  ProfScope prof((flags & SR3D_PROFILE) && !(flags & SR3D_USE_GRAPH));

  // Host images of the descriptors and items.
  std::vector<RowDesc> r2c(count), c2r(count);
  std::vector<StridedDesc> fn(count), in_(count), fs(count), is(count);
  std::vector<FoldArgs> fold(count);
  std::vector<SolveSArgs> solv(count);
  std::vector<BatchStencilDesc> sten(count);
  std::vector<ReduceDesc> red(count);
  std::vector<float *> nu0(count);
  for (int v = 0; v < count; ++v) {
    const Geometry &G = g[v];
    const TvWs &L = Ls[v];
    const int *done = &L.ctrl->done;
    const long Mh = G.Mh;
    nu0[v] = p[v].state ? p[v].state : L.nu[0];
    const int *kofp = L.fused ? L.tab : nullptr, *posk = L.fused ? L.tab + G.Mh : nullptr;
    float2 *xs = L.fused ? L.w : L.w2;  // spectrum of the x-update
    const long P = L.fused ? G.sp.pitch : Mh;  // spectrum row pitch
    r2c[v] = RowDesc{L.theta, L.w, nullptr, (long)G.S * G.N, 1.0f, done, kofp, posk, (int)P,
                     RedArgs{}};
    c2r[v] = RowDesc{nullptr, xs, p[v].x, (long)G.S * G.N, 1.0f, done, kofp, posk, (int)P,
                     RedArgs{}};
    fn[v] = make_strided_desc(L.w, (long)G.S * P, P, (long)G.N * P, P, done, Mh);
    in_[v] = make_strided_desc(xs, (long)G.S * P, P, (long)G.N * P, P, done, Mh);
    fs[v] = make_strided_desc(L.w, (long)G.N * Mh, (long)G.N * Mh, 0, (long)G.N * Mh, done);
    is[v] = make_strided_desc(L.w2, (long)G.N * Mh, (long)G.N * Mh, 0, (long)G.N * Mh, done);
    FoldArgs fa = make_fold(G);
    fa.W = L.w; fa.Lam = L.lam; fa.Yh = L.yh; fa.X = L.w2;
    fa.gm = L.g; fa.gn = L.g + G.M; fa.gs = L.g + G.M + G.N;
    fa.cw = p[v].mu; fa.coefA = p[v].mu; fa.tv = 1;
    fa.partial = L.partF; fa.ctrl = L.ctrl; fa.done = done;
    fold[v] = fa;
    if (L.fused) solv[v] = make_solve_args(G, L, &p[v]);
    BatchStencilDesc sd{};
    sd.a.x = p[v].x; sd.a.theta = L.theta;
    sd.a.S = G.S; sd.a.N = G.N; sd.a.M = G.M; sd.a.thr = p[v].lambda_tv / p[v].mu;
    sd.a.part = L.partS; sd.a.done = done; sd.a.aniso = L.aniso ? 1 : 0;
    sd.nu[0] = nu0[v];
    sd.nu[1] = L.nu[1];
    sd.pl = L.fsten ? stencil_r2c_plan(G.S, G.N, G.M) : stencil_plan(G.S, G.N, G.M);
    sd.spec = L.w;
    sd.kofp = L.tab;
    sd.pitch = G.sp.pitch;
    sten[v] = sd;
    red[v] = ReduceDesc{L.ctrl, L.partS, L.nbS, L.partF, L.nbF};
  }
  std::vector<int2> items;
  items.reserve(nitems);
  for (auto &gr : plan.groups) {
    gr.off = items.size() * sizeof(int2);
    items.insert(items.end(), gr.items.begin(), gr.items.end());
  }
  std::vector<char> himg(hdr, 0);
  auto put = [&](void *dst, const void *src, size_t bytes) {
    memcpy(himg.data() + (reinterpret_cast<char *>(dst) - base), src, bytes);
  };
  put(H.r2c, r2c.data(), sizeof(RowDesc) * count);
  put(H.c2r, c2r.data(), sizeof(RowDesc) * count);
  put(H.fn, fn.data(), sizeof(StridedDesc) * count);
  put(H.in_, in_.data(), sizeof(StridedDesc) * count);
  put(H.fs, fs.data(), sizeof(StridedDesc) * count);
  put(H.is, is.data(), sizeof(StridedDesc) * count);
  put(H.fold, fold.data(), sizeof(FoldArgs) * count);
  put(H.solve, solv.data(), sizeof(SolveSArgs) * count);
  put(H.sten, sten.data(), sizeof(BatchStencilDesc) * count);
  put(H.red, red.data(), sizeof(ReduceDesc) * count);
  int active0 = count;
  put(H.active, &active0, sizeof(int));
  if (!items.empty()) put(H.items, items.data(), sizeof(int2) * items.size());
  SR3D_TRY(hipMemcpyAsync(base, himg.data(), hdr, hipMemcpyHostToDevice, st), "batch header");

  t_prof.override_stage = prof.on ? kStSetup : -1;
  for (int v = 0; v < count; ++v) SR3D_TRY(tv_setup(g[v], Ls[v], &p[v], nu0[v], flags, st), "batch setup");
  t_prof.override_stage = -1;
  int max_iter = 0;
  for (int v = 0; v < count; ++v) max_iter = p[v].max_iter > max_iter ? p[v].max_iter : max_iter;

  int K = check_interval(flags);
  int *h_active = reinterpret_cast<int *>(hc);
  if (flags & SR3D_USE_GRAPH) {
    K += K & 1;
    hipStream_t cs;
    SR3D_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream create");
    hipEvent_t ev;
    SR3D_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    for (int i = 1; e == hipSuccess && i <= K; ++i)
      e = batch_iteration(plan, H, g, Ls, p, i, fp64, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    for (int it = 0; e == hipSuccess && it < max_iter; it += K) {
      e = hipGraphLaunch(exec, cs);
      if (e == hipSuccess) e = hipMemcpyAsync(h_active, H.active, sizeof(int), hipMemcpyDeviceToHost, cs);
      if (e == hipSuccess) e = hipStreamSynchronize(cs);
      if (e == hipSuccess && *h_active <= 0) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipEventRecord(ev, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    (void)hipStreamSynchronize(cs);
    (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "batch graph replay");
  } else {
    for (int it = 0; it < max_iter;) {
      const int n = (max_iter - it) < K ? (max_iter - it) : K;
      for (int i = 1; i <= n; ++i)
        SR3D_TRY(batch_iteration(plan, H, g, Ls, p, it + i, fp64, st), "batch iteration");
      it += n;
      SR3D_TRY(hipMemcpyAsync(h_active, H.active, sizeof(int), hipMemcpyDeviceToHost, st), "active copy");
      SR3D_TRY(hipStreamSynchronize(st), "stream sync");
      if (prof.on) prof_flush();
      if (*h_active <= 0) break;
    }
  }
  // Per-volume results.
  int status = SR3D_OK;
  for (int v = 0; v < count; ++v) {
    SR3D_TRY(hipMemcpyAsync(hc, Ls[v].ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st), "ctrl copy");
    SR3D_TRY(hipStreamSynchronize(st), "stream sync");
    if (stats) {
      stats[v].iters = hc->iter;
      stats[v].converged = hc->converged;
      stats[v].primal_rel = hc->primal_rel;
      stats[v].dual_rel = hc->dual_rel;
      stats[v].objective = hc->objective;
    }
    if (hc->status && !status) status = hc->status;
    if (p[v].state && (hc->iter & 1)) {
      SR3D_TRY(hipMemcpyAsync(p[v].state, Ls[v].nu[1], sizeof(float) * 3 * (size_t)g[v].NH,
                              hipMemcpyDeviceToDevice, st), "state copy");
    }
  }
  SR3D_TRY(hipStreamSynchronize(st), "stream sync");
  if (status)
    return fail(status, status == SR3D_ERR_SINGULAR ? "Lambda(0) = 0 in a batch volume"
                                                    : "non-finite residual in a batch volume");
  return SR3D_OK;
}

int check_tikhonov(sr3d_dims hr, sr3d_rate rate, const float *y, const float *psf,
                   sr3d_dims psf_dims, const float *xbar, float lambda, const float *x,
                   Geometry *g) {
  int rc = check_geometry(hr, rate, &psf_dims, g);
  if (rc) return rc;
  if (!y || !psf || !x) return fail(SR3D_ERR_INVALID_ARG, "y, psf and x must be non-NULL");
  if (!(lambda > 0.f) || !isfinite(lambda)) return fail(SR3D_ERR_INVALID_ARG, "lambda must be finite and > 0");
  if (x == y || x == psf || (xbar && x == xbar)) return fail(SR3D_ERR_INVALID_ARG, "x aliases an input");
  return SR3D_OK;
}

// eq. (12): Lambda and Y by R2C, the per-group solve with A = 2 lambda and
// K = conj(Lambda) Y + 2 lambda F xbar, one C2R. Every workspace buffer is
// written before it is read, so nothing needs clearing.
int tikhonov_run(const Geometry &g, const TikWs &L, const float *y, const float *psf,
                 sr3d_dims psf_dims, const float *xbar, float lambda, float *x, hipStream_t st) {
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(pad_psf(psf, psf_dims.s, psf_dims.n, psf_dims.m, L.real, g.S, g.N, g.M, st), "pad psf");
  SR3D_TRY(fft3d_forward(L.real, L.lam, g.S, g.N, g.M, nullptr, st), "fft Lambda");
  SR3D_TRY(fft3d_forward(y, L.yh, g.Sl, g.Nl, g.Ml, nullptr, st), "fft y");
  if (xbar) SR3D_TRY(fft3d_forward(xbar, L.w, g.S, g.N, g.M, nullptr, st), "fft xbar");
  FoldArgs fa = make_fold(g);
  fa.W = xbar ? L.w : nullptr; fa.Lam = L.lam; fa.Yh = L.yh; fa.X = L.w2;
  fa.cw = 2.0f * lambda; fa.coefA = 2.0f * lambda; fa.tv = 0;
  fa.partial = nullptr; fa.ctrl = nullptr; fa.done = nullptr;
  SR3D_TRY(fold_solve(fa, false, st), "fold solve");
  SR3D_TRY(fft3d_inverse(L.w2, x, g.S, g.N, g.M, 1.0f, nullptr, st), "inverse fft");
  return SR3D_OK;
}

std::mutex g_scratch_mu;
char *g_scratch[64] = {nullptr};

hipError_t scratch_address(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = reinterpret_cast<char *>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// PSF fit workspace: the HR half spectrum of x, the LR half spectrum of y,
// the per-axis kernel tables, the per-workgroup partial sums and the totals.
struct PsfWs {
  float2 *X, *Yh;
  float *tab;
  double *part, *out;
};

size_t psf_fit_layout(const Geometry &g, char *base, PsfWs *L) {
  Carve c{base, 0};
  PsfWs tmp;
  PsfWs *w = L ? L : &tmp;
  w->X = c.take<float2>(g.nspec);
  w->Yh = c.take<float2>(g.nlspec);
  w->tab = c.take<float>((size_t)2 * (g.M + g.N + g.S));
  w->part = c.take<double>((size_t)psf_fit_nsums() * psf_fit_blocks(g.nlspec));
  w->out = c.take<double>((size_t)psf_fit_nsums());
  return c.off + 256;
}

// DFT of the symmetric sampled Gaussian g_i = exp(-i^2/(2 s^2)) / sum
// (|i| <= R, wrapped onto a circle of n points) and its derivative with
// respect to s, in FP64: l(k) = sum_i g_i cos(2 pi k i / n),
// dg_i/ds = g_i (i^2 - E[j^2]) / s^3.
void gaussian_dft(int n, double s, int R, float *l, float *dl) {
  std::vector<double> g(2 * R + 1);
  double W = 0.0, m2 = 0.0;
  for (int i = -R; i <= R; ++i) {
    g[i + R] = exp(-(double)i * i / (2.0 * s * s));
    W += g[i + R];
  }
  for (int i = -R; i <= R; ++i) {
    g[i + R] /= W;
    m2 += g[i + R] * i * i;
  }
  for (int k = 0; k < n; ++k) {
    double a = 0.0, b = 0.0;
    for (int i = -R; i <= R; ++i) {
      const long ki = ((long)k * i) % n;
      const double cs = cos(2.0 * M_PI * (double)ki / (double)n);
      a += g[i + R] * cs;
      b += g[i + R] * ((double)i * i - m2) / (s * s * s) * cs;
    }
    l[k] = (float)a;
    dl[k] = (float)b;
  }
}

// Solves the n x n system A z = b (n <= 4) by Gaussian elimination with
// partial pivoting; false if singular.
bool solve_small(int n, const double A[4][4], const double *b, double *z) {
  double M[4][5];
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) M[i][j] = A[i][j];
    M[i][n] = b[i];
  }
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
    if (!(fabs(M[p][c]) > 0.0)) return false;
    for (int j = 0; j <= n; ++j) std::swap(M[c][j], M[p][j]);
    for (int r = c + 1; r < n; ++r) {
      const double f = M[r][c] / M[c][c];
      for (int j = c; j <= n; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = M[i][n];
    for (int j = i + 1; j < n; ++j) t -= M[i][j] * z[j];
    z[i] = t / M[i][i];
  }
  return true;
}

}  // namespace

extern "C" {

size_t sr3d_workspace_size(int op, const sr3d_problem *p, int count) {
  if (!p || count < 1) return 0;
  if (op == SR3D_OP_BATCH) {
    std::vector<Geometry> gs;
    std::vector<size_t> offs;
    BatchPlan plan;
    size_t hdr = 0;
    return batch_workspace(p, count, 0, &gs, &offs, &plan, &hdr);
  }
  Geometry g;
  size_t total = 0;
  const int n = (op == SR3D_OP_BATCH) ? count : 1;
  for (int i = 0; i < n; ++i) {
    const sr3d_dims *psf = (op == SR3D_OP_FFT || op == SR3D_OP_PSF_FIT) ? nullptr : &p[i].psf_dims;
    sr3d_rate r = p[i].rate;
    if (op == SR3D_OP_FFT) r = sr3d_rate{1, 1, 1};
    if (check_geometry(p[i].hr, r, psf, &g) != SR3D_OK) return 0;
    TvWs tv;
    TikWs tk;
    size_t b = 0;
    switch (op) {
      case SR3D_OP_TIKHONOV: b = tik_layout(g, nullptr, &tk); break;
      case SR3D_OP_TV_ADMM:
      case SR3D_OP_BATCH: b = tv_layout(g, nullptr, &tv); break;
      case SR3D_OP_DEGRADE: b = degrade_layout(g, nullptr, &tk); break;
      case SR3D_OP_FFT: b = 0; break;
      case SR3D_OP_PSF_FIT: b = psf_fit_layout(g, nullptr, nullptr); break;
      case SR3D_OP_TIKHONOV_MF:
        if (count < 1 || count > kMaxFrames) return 0;
        b = tik_layout(g, nullptr, &tk) + mf_extra(g, count);
        break;
      case SR3D_OP_TV_ADMM_MF:
        if (count < 1 || count > kMaxFrames) return 0;
        b = tv_layout(g, nullptr, &tv) + mf_extra(g, count);
        break;
      default: return 0;
    }
    if (op == SR3D_OP_BATCH) total = b > total ? b : total;
    else total += b;
  }
  return total;
}

int sr3d_tikhonov(sr3d_dims hr, sr3d_rate rate, const float *y, const float *psf, sr3d_dims psf_dims,
                  const float *xbar, float lambda, float *x, void *ws, size_t ws_bytes,
                  hipStream_t st) {
  Geometry g;
  int rc = check_tikhonov(hr, rate, y, psf, psf_dims, xbar, lambda, x, &g);
  if (rc) return rc;
  TikWs L;
  const size_t need = tik_layout(g, nullptr, &L);
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  tik_layout(g, reinterpret_cast<char *>(ws), &L);
  return tikhonov_run(g, L, y, psf, psf_dims, xbar, lambda, x, st);
}

int sr3d_tikhonov_noalloc(sr3d_dims hr, sr3d_rate rate, const float *y, const float *psf,
                          sr3d_dims psf_dims, const float *xbar, float lambda, float *x,
                          hipStream_t st) {
  Geometry g;
  int rc = check_tikhonov(hr, rate, y, psf, psf_dims, xbar, lambda, x, &g);
  if (rc) return rc;
  TikWs L;
  if (tik_layout(g, nullptr, &L) > sizeof(scratch))
    return fail(SR3D_ERR_WORKSPACE, "problem needs more than the " +
                                        std::to_string(sizeof(scratch) >> 20) +
                                        " MiB static scratch of sr3d_tikhonov_noalloc");
  char *base = nullptr;
  SR3D_TRY(scratch_address(&base), "static scratch address");
  tik_layout(g, base, &L);
  return tikhonov_run(g, L, y, psf, psf_dims, xbar, lambda, x, st);
}

int sr3d_tv_admm(const sr3d_problem *p, int flags, sr3d_stats *stats, void *ws, size_t ws_bytes,
                 hipStream_t st) {
  return run_tv(p, flags, stats, ws, ws_bytes, st);
}

int sr3d_tv_admm_mf(const sr3d_problem *p, int nframes, const float *const *y, const int *shifts,
                    int flags, sr3d_stats *stats, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p) return fail(SR3D_ERR_INVALID_ARG, "problem is NULL");
  if (!y || nframes < 1) return fail(SR3D_ERR_INVALID_ARG, "frames must be non-NULL");
  sr3d_problem q = *p;
  q.y = y[0];  // the single-frame checks; the frames themselves are read below
  return run_tv(&q, flags, stats, ws, ws_bytes, st, nframes, y, shifts);
}

int sr3d_tikhonov_mf(sr3d_dims hr, sr3d_rate rate, int nframes, const float *const *y,
                     const int *shifts, const float *psf, sr3d_dims psf_dims, const float *xbar,
                     float lambda, float *x, void *ws, size_t ws_bytes, hipStream_t st) {
  Geometry g;
  int rc = check_tikhonov(hr, rate, (y && nframes > 0) ? y[0] : nullptr, psf, psf_dims, xbar,
                          lambda, x, &g);
  if (rc) return rc;
  if ((rc = check_frames(g, nframes, y, shifts))) return rc;
  for (int f = 0; f < nframes; ++f)
    if (x == y[f]) return fail(SR3D_ERR_INVALID_ARG, "x aliases an input");
  TikWs L;
  const size_t base_need = tik_layout(g, nullptr, &L);
  const size_t need = base_need + mf_extra(g, nframes);
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  tik_layout(g, reinterpret_cast<char *>(ws), &L);
  float2 *yf = reinterpret_cast<float2 *>(reinterpret_cast<char *>(ws) + base_need);
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(pad_psf(psf, psf_dims.s, psf_dims.n, psf_dims.m, L.real, g.S, g.N, g.M, st), "pad psf");
  SR3D_TRY(fft3d_forward(L.real, L.lam, g.S, g.N, g.M, nullptr, st), "fft Lambda");
  for (int f = 0; f < nframes; ++f)
    SR3D_TRY(fft3d_forward(y[f], yf + (size_t)f * g.nlspec, g.Sl, g.Nl, g.Ml, nullptr, st),
             "frame spectra");
  if (xbar) SR3D_TRY(fft3d_forward(xbar, L.w, g.S, g.N, g.M, nullptr, st), "fft xbar");
  int t[kMaxFrames][3];
  for (int f = 0; f < nframes; ++f)
    for (int c = 0; c < 3; ++c) t[f][c] = shifts[3 * f + c];
  MfArgs ma = make_mf(g, L.lam, yf, nframes, t);
  ma.W = xbar ? L.w : nullptr; ma.X = L.w2;
  ma.cw = 2.0f * lambda; ma.coefA = 2.0f * lambda; ma.tv = 0;
  SR3D_TRY(fold_solve_mf(ma, false, st), "multi-frame fold solve");
  SR3D_TRY(fft3d_inverse(L.w2, x, g.S, g.N, g.M, 1.0f, nullptr, st), "inverse fft");
  return SR3D_OK;
}

int sr3d_batch(const sr3d_problem *p, int count, int flags, sr3d_stats *stats, void *ws,
               size_t ws_bytes, hipStream_t st) {
  return run_batch(p, count, flags, stats, ws, ws_bytes, st);
}

int sr3d_degrade(sr3d_dims hr, sr3d_rate rate, const float *x, const float *psf, sr3d_dims psf_dims,
                 float *y, void *ws, size_t ws_bytes, hipStream_t st) {
  Geometry g;
  int rc = check_geometry(hr, rate, &psf_dims, &g);
  if (rc) return rc;
  if (!x || !psf || !y) return fail(SR3D_ERR_INVALID_ARG, "x, psf and y must be non-NULL");
  TikWs L;
  const size_t need = degrade_layout(g, nullptr, &L);
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  degrade_layout(g, reinterpret_cast<char *>(ws), &L);
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(pad_psf(psf, psf_dims.s, psf_dims.n, psf_dims.m, L.real, g.S, g.N, g.M, st), "pad psf");
  SR3D_TRY(fft3d_forward(L.real, L.lam, g.S, g.N, g.M, nullptr, st), "fft Lambda");
  SR3D_TRY(fft3d_forward(x, L.w, g.S, g.N, g.M, nullptr, st), "fft x");
  SR3D_TRY(spectrum_mul(L.w, L.lam, (size_t)g.nspec, (float)(1.0 / (double)g.NH), st), "multiply");
  SR3D_TRY(fft3d_inverse(L.w, L.real, g.S, g.N, g.M, 1.0f, nullptr, st), "inverse fft");
  SR3D_TRY(decimate(L.real, y, g.S, g.N, g.M, g.dr, g.dc, g.ds, st), "decimate");
  return SR3D_OK;
}

int sr3d_psf_fit(sr3d_dims hr, sr3d_rate rate, const float *x, const float *y, const int radius[3],
                 const double sigma0[3], int max_iter, double tol, sr3d_psf_fit_result *res,
                 void *ws, size_t ws_bytes, hipStream_t st) {
  Geometry g;
  int rc = check_geometry(hr, rate, nullptr, &g);
  if (rc) return rc;
  if (!x || !y || !radius || !sigma0 || !res) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  for (int a = 0; a < 3; ++a) {
    if (radius[a] < 0 || radius[a] > 4096) return fail(SR3D_ERR_INVALID_ARG, "radius out of range");
    if (!(sigma0[a] > 0.0) || !isfinite(sigma0[a]))
      return fail(SR3D_ERR_INVALID_ARG, "sigma0 must be finite and > 0");
  }
  if (max_iter < 1 || !(tol >= 0.0)) return fail(SR3D_ERR_INVALID_ARG, "max_iter >= 1, tol >= 0");
  if (g.NL < 2) return fail(SR3D_ERR_INVALID_ARG, "the LR volume needs more than one voxel");
  PsfWs L;
  const size_t need = psf_fit_layout(g, nullptr, nullptr);
  if (!ws || ws_bytes < need) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  psf_fit_layout(g, reinterpret_cast<char *>(ws), &L);
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(fft3d_forward(x, L.X, g.S, g.N, g.M, nullptr, st), "fft x");
  SR3D_TRY(fft3d_forward(y, L.Yh, g.Sl, g.Nl, g.Ml, nullptr, st), "fft y");
  float2 y0;
  SR3D_TRY(hipMemcpyAsync(&y0, L.Yh, sizeof y0, hipMemcpyDeviceToHost, st), "copy Y0");
  const int n_ax[3] = {g.M, g.N, g.S};
  const int ntab = g.M + g.N + g.S;
  std::vector<float> tab((size_t)2 * ntab);
  double sums[17];
  int passes = 0;
  // One pass: f, the Gauss-Newton matrix and right-hand side at theta.
  auto evaluate = [&](const double *th, double *f, double G[4][4], double *bv) -> hipError_t {
    int off = 0;
    for (int a = 0; a < 3; ++a) {
      gaussian_dft(n_ax[a], th[a], radius[a], tab.data() + off, tab.data() + ntab + off);
      off += n_ax[a];
    }
    hipError_t e = hipMemcpyAsync(L.tab, tab.data(), sizeof(float) * tab.size(),
                                  hipMemcpyHostToDevice, st);
    if (!e) e = psf_fit_sums(L.X, L.Yh, L.tab, (float)th[3], g.S, g.N, g.M, g.dr, g.dc, g.ds,
                             L.part, L.out, st);
    if (!e) e = hipMemcpyAsync(sums, L.out, sizeof sums, hipMemcpyDeviceToHost, st);
    if (!e) e = hipStreamSynchronize(st);
    if (e) return e;
    ++passes;
    const double inl = 1.0 / (double)g.NL;
    int q = 0;
    for (int u = 0; u < 4; ++u)
      for (int v = u; v < 4; ++v) G[u][v] = G[v][u] = sums[q++] * inl;
    for (int u = 0; u < 4; ++u) bv[u] = sums[10 + u] * inl;
    *f = 0.5 * sums[14] * inl;
    return hipSuccess;
  };
  // theta = (sigma_m, sigma_n, sigma_s, alpha); alpha starts at its
  // least-squares value for sigma0 (from a pass at alpha = 1, where
  // Re(m^H Y) = Jtr_alpha + JtJ_alpha,alpha).
  double th[4] = {sigma0[0], sigma0[1], sigma0[2], 1.0};
  double f, G[4][4], bv[4];
  SR3D_TRY(evaluate(th, &f, G, bv), "psf fit pass");
  if (G[3][3] > 0.0) th[3] = (bv[3] + G[3][3]) / G[3][3];
  SR3D_TRY(evaluate(th, &f, G, bv), "psf fit pass");
  double m0 = sums[15];  // real part of m_0 at the accepted theta
  // Levenberg-Marquardt on the Gauss-Newton model.
  double lam = 1e-3;
  bool converged = false;
  for (int it = 0; it < max_iter && !converged; ++it) {
    bool stepped = false;
    for (int tries = 0; tries < 12 && !stepped && !converged; ++tries) {
      double A[4][4], z[4], tn[4], fn, Gn[4][4], bn[4];
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) A[u][v] = G[u][v] + (u == v ? lam * G[u][u] : 0.0);
      if (!solve_small(4, A, bv, z)) {
        lam *= 10.0;
        continue;
      }
      double step = 0.0;
      for (int u = 0; u < 4; ++u) {
        tn[u] = th[u] + z[u];
        if (u < 3 && tn[u] < 0.05) tn[u] = 0.05;
        step = fmax(step, fabs(tn[u] - th[u]) / fmax(fabs(th[u]), 1e-3));
      }
      SR3D_TRY(evaluate(tn, &fn, Gn, bn), "psf fit pass");
      if (fn <= f) {
        const double df = f - fn;
        for (int u = 0; u < 4; ++u) {
          th[u] = tn[u];
          bv[u] = bn[u];
          for (int v = 0; v < 4; ++v) G[u][v] = Gn[u][v];
        }
        f = fn;
        m0 = sums[15];
        lam = fmax(lam / 3.0, 1e-12);
        stepped = true;
        if (step <= tol || df <= 1e-15 * fn) converged = true;
      } else {
        lam *= 4.0;
        // no decrease from a step below the tolerance: at the minimum
        if (step <= tol) converged = true;
      }
    }
    if (!stepped) break;
  }
  // The offset that zeroes the zero-frequency residual: beta = (Y_0 - alpha m_0) / N_l.
  for (int a = 0; a < 3; ++a) res->sigma[a] = th[a];
  res->gain = th[3];
  res->offset = ((double)y0.x - th[3] * m0) / (double)g.NL;
  res->objective = f;
  res->passes = passes;
  res->converged = converged ? 1 : 0;
  return SR3D_OK;
}

int sr3d_rfft3d(sr3d_dims d, const float *in, float *spec, hipStream_t st) {
  Geometry g;
  int rc = check_geometry(d, sr3d_rate{1, 1, 1}, nullptr, &g);
  if (rc) return rc;
  if (!in || !spec) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(fft3d_forward(in, reinterpret_cast<float2 *>(spec), g.S, g.N, g.M, nullptr, st), "rfft3d");
  return SR3D_OK;
}

int sr3d_irfft3d(sr3d_dims d, float *spec, float *out, hipStream_t st) {
  Geometry g;
  int rc = check_geometry(d, sr3d_rate{1, 1, 1}, nullptr, &g);
  if (rc) return rc;
  if (!spec || !out) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  SR3D_TRY(ensure_device_tables(), "twiddle tables");
  SR3D_TRY(fft3d_inverse(reinterpret_cast<float2 *>(spec), out, g.S, g.N, g.M,
                         (float)(1.0 / (double)g.NH), nullptr, st),
           "irfft3d");
  return SR3D_OK;
}

const char *sr3d_status_string(int s) {
  switch (s) {
    case SR3D_OK: return "SR3D_OK";
    case SR3D_ERR_INVALID_ARG: return "SR3D_ERR_INVALID_ARG";
    case SR3D_ERR_NOT_DIVISIBLE: return "SR3D_ERR_NOT_DIVISIBLE";
    case SR3D_ERR_PSF_TOO_LARGE: return "SR3D_ERR_PSF_TOO_LARGE";
    case SR3D_ERR_UNSUPPORTED_SIZE: return "SR3D_ERR_UNSUPPORTED_SIZE";
    case SR3D_ERR_WORKSPACE: return "SR3D_ERR_WORKSPACE";
    case SR3D_ERR_SINGULAR: return "SR3D_ERR_SINGULAR";
    case SR3D_ERR_NONFINITE: return "SR3D_ERR_NONFINITE";
    case SR3D_ERR_HIP: return "SR3D_ERR_HIP";
    default: return "SR3D_ERR_UNKNOWN";
  }
}

const char *sr3d_last_error(void) { return g_err.c_str(); }

static int check_cnn_dims(sr3d_dims d, long *NV) {
  if (d.m < 1 || d.n < 1 || d.s < 1) return fail(SR3D_ERR_INVALID_ARG, "dimensions must be >= 1");
  const long nv = (long)d.m * d.n * d.s;
  if (nv >= (1L << 31)) return fail(SR3D_ERR_UNSUPPORTED_SIZE, "volume too large");
  *NV = nv;
  return SR3D_OK;
}

size_t sr3d_cnn_param_count(void) { return (size_t)cnn_param_count(); }

int sr3d_cnn_init(float *params, unsigned long long seed, hipStream_t st) {
  if (!params) return fail(SR3D_ERR_INVALID_ARG, "params is NULL");
  SR3D_TRY(cnn_init(params, seed, st), "cnn init");
  return SR3D_OK;
}

size_t sr3d_cnn_workspace_size(sr3d_dims d, int training) {
  long nv;
  if (check_cnn_dims(d, &nv)) return 0;
  return cnn_layout(d.s, d.n, d.m, training != 0, nullptr).bytes;
}

int sr3d_cnn_forward(sr3d_dims d, const float *params, const float *x, float *y, void *ws,
                     size_t ws_bytes, hipStream_t st) {
  long nv;
  int rc = check_cnn_dims(d, &nv);
  if (rc) return rc;
  if (!params || !x || !y) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  if (x == y) return fail(SR3D_ERR_INVALID_ARG, "y aliases x");
  const CnnWs L0 = cnn_layout(d.s, d.n, d.m, false, nullptr);
  if (!ws || ws_bytes < L0.bytes) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  const CnnWs L = cnn_layout(d.s, d.n, d.m, false, reinterpret_cast<char *>(ws));
  SR3D_TRY(cnn_forward(d.s, d.n, d.m, params, x, y, L, false, nullptr, nullptr, nullptr, st),
           "cnn forward");
  return SR3D_OK;
}

int sr3d_cnn_grad(sr3d_dims d, const float *params, const float *x, const float *target,
                  float *grad, float *loss, void *ws, size_t ws_bytes, hipStream_t st) {
  long nv;
  int rc = check_cnn_dims(d, &nv);
  if (rc) return rc;
  if (!params || !x || !target || !grad || !loss) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  const CnnWs L0 = cnn_layout(d.s, d.n, d.m, true, nullptr);
  if (!ws || ws_bytes < L0.bytes) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  const CnnWs L = cnn_layout(d.s, d.n, d.m, true, reinterpret_cast<char *>(ws));
  SR3D_TRY(cnn_grad(d.s, d.n, d.m, params, x, target, grad, loss, L, st), "cnn grad");
  return SR3D_OK;
}

int sr3d_cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                  float beta1, float beta2, float eps, hipStream_t st) {
  if (!params || !grad || !m || !v) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(SR3D_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  SR3D_TRY(cnn_adam(params, grad, m, v, step, lr, beta1, beta2, eps, st), "adam");
  return SR3D_OK;
}

size_t sr3d_conv3d_workspace_size(sr3d_dims d) {
  long nv;
  if (check_cnn_dims(d, &nv)) return 0;
  return 256 + ((27 * 32 * 32 * sizeof(uint16_t) + 255) & ~(size_t)255) + conv_layer_partial_bytes(nv);
}

int sr3d_conv3d_forward(sr3d_dims d, int cin, int cout, const void *in_bf16, const float *x,
                        const float *weight, const float *bias, void *out_bf16, float *out_f32,
                        void *ws, size_t ws_bytes, hipStream_t st) {
  long nv;
  int rc = check_cnn_dims(d, &nv);
  if (rc) return rc;
  if (!((cin == 1 && cout == 32 && x) || (cin == 32 && cout == 32 && in_bf16)))
    return fail(SR3D_ERR_INVALID_ARG, "supported layers: 1->32 (x) and 32->32 (in_bf16)");
  if (!weight || !bias || !out_bf16) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  if (!ws || ws_bytes < sr3d_conv3d_workspace_size(d)) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  uint16_t *wbf = reinterpret_cast<uint16_t *>(ws);
  SR3D_TRY(to_bf16(weight, wbf, 27L * cin * cout, st), "weights to bf16");
  SR3D_TRY(conv_layer_forward(d.s, d.n, d.m, cin, cout, in_bf16, x, wbf, bias, out_bf16, out_f32, st),
           "conv forward");
  return SR3D_OK;
}

int sr3d_conv3d_backward(sr3d_dims d, const void *act_in_bf16, const void *gout_bf16,
                         const float *weight, const void *mask_bf16, void *gin_bf16,
                         float *gin_f32, float *gweight, void *ws, size_t ws_bytes,
                         hipStream_t st) {
  long nv;
  int rc = check_cnn_dims(d, &nv);
  if (rc) return rc;
  if (!act_in_bf16 || !gout_bf16 || !weight || !gweight) return fail(SR3D_ERR_INVALID_ARG, "NULL pointer");
  if (gin_bf16 && !mask_bf16) return fail(SR3D_ERR_INVALID_ARG, "input gradient needs a mask");
  if (!ws || ws_bytes < sr3d_conv3d_workspace_size(d)) return fail(SR3D_ERR_WORKSPACE, "workspace too small");
  uint16_t *wbf = reinterpret_cast<uint16_t *>(ws);
  float *partial = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) +
                                             ((27 * 32 * 32 * sizeof(uint16_t) + 255) & ~(size_t)255));
  SR3D_TRY(to_bf16(weight, wbf, 27L * 32 * 32, st), "weights to bf16");
  SR3D_TRY(conv_layer_backward(d.s, d.n, d.m, act_in_bf16, gout_bf16, wbf, mask_bf16, gin_bf16,
                               gin_f32, gweight, partial, st),
           "conv backward");
  return SR3D_OK;
}

int sr3d_autotune(const sr3d_problem *p, int count, int force, hipStream_t st) {
  if (!p || count < 1) return fail(SR3D_ERR_INVALID_ARG, "no problems");
  Geometry g;
  for (int i = 0; i < count; ++i) {
    int rc = check_geometry(p[i].hr, p[i].rate, &p[i].psf_dims, &g);
    if (rc) return rc;
  }
  for (int i = 0; i < count; ++i) {
    check_geometry(p[i].hr, p[i].rate, &p[i].psf_dims, &g);
    // the m and n passes are timed in the layout the solver runs them in
    SR3D_TRY(fft_autotune(g.S, g.N, g.M, g.sp.fused ? g.sp.pitch : 0, force != 0, st),
             "autotune HR");
    SR3D_TRY(fft_autotune(g.Sl, g.Nl, g.Ml, 0, force != 0, st), "autotune LR");
  }
  return SR3D_OK;
}

int sr3d_tune_save(const char *path) {
  if (!path || fft_tune_save(path) != 0) return fail(SR3D_ERR_INVALID_ARG, "cannot write tune file");
  return SR3D_OK;
}

int sr3d_tune_load(const char *path) {
  if (!path) return fail(SR3D_ERR_INVALID_ARG, "NULL path");
  const int n = fft_tune_load(path);
  if (n < 0) return fail(SR3D_ERR_INVALID_ARG, "cannot read tune file");
  return n;
}

int sr3d_profile_read(int stage, const char **name, double *total_ms, long *launches) {
  if (stage < 0 || stage >= kStCount) return SR3D_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (name) *name = kStageNames[stage];
  if (total_ms) *total_ms = g_prof_ms[stage];
  if (launches) *launches = g_prof_n[stage];
  return SR3D_OK;
}

void sr3d_profile_select(unsigned stage_mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mask = stage_mask;
}

void sr3d_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < kStCount; ++i) {
    g_prof_ms[i] = 0.0;
    g_prof_n[i] = 0;
  }
}

void sr3d_shutdown(void) {
  release_device_tables();
  std::lock_guard<std::mutex> lk(g_host_mu);
  for (Ctrl *c : g_host_blocks) (void)hipHostFree(c);
  g_host_blocks.clear();
  t_host_ctrl = nullptr;
}

}  // extern "C"
