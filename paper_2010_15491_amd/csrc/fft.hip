// 3D FFT orchestration for gfx950: one launch per axis (m: R2C/C2R, n and s:
// strided C2C in place), per-device twiddle tables, and the tile-size
// autotuner.
//
// The paper needs one forward and one inverse 3D DFT per x-update (eq. (12)
// and Algorithm 1 step 5a). Every axis kernel stages T lines in LDS and runs
// Stockham radix-8/4/3/2 passes there (fft_core.h); T follows from the tile
// size (2048, 4096 or 8192 complex elements) chosen per (axis kind, length),
// by default or by timing every variant on the device (sr3d_autotune).
// Twiddles are computed once per device in FP64 and rounded to FP32.
#include <math.h>
#include <stdio.h>

#include <mutex>
#include <vector>

#include "fft_core.h"

namespace sr3d {

// ---------------------------------------------------------------------------
// Twiddle tables (per device)
// ---------------------------------------------------------------------------

bool fft_len_supported(int n) {
  switch (n) {
#define SR3D_CASE(L) case L:
    case 1:
    SR3D_FFT_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
      return true;
    default:
      return false;
  }
}

namespace {
constexpr int kMaxDev = 64;

// Total entries of all tables: sum of the supported lengths (and length 1).
constexpr int tw_total() {
  int t = 1;
#define SR3D_SUM(L) t += L;
  SR3D_FFT_LENGTHS(SR3D_SUM)
#undef SR3D_SUM
  return t;
}
constexpr int kTwTotal = tw_total();

std::mutex g_mu;
float2 *g_tw[kMaxDev] = {nullptr};
int g_tw_off[kMaxLen + 1];
bool g_off_ready = false;
float2 g_tw_host[kTwTotal];

void build_offsets() {
  if (g_off_ready) return;
  int off = 0;
  for (int n = 0; n <= kMaxLen; ++n) g_tw_off[n] = -1;
#define SR3D_OFF(L) g_tw_off[L] = off; off += L;
  SR3D_OFF(1)
  SR3D_FFT_LENGTHS(SR3D_OFF)
#undef SR3D_OFF
  for (int n = 1; n <= kMaxLen; ++n) {
    if (g_tw_off[n] < 0) continue;
    for (int k = 0; k < n; ++k) {
      const double a = -2.0 * M_PI * (double)k / (double)n;
      g_tw_host[g_tw_off[n] + k] = make_float2((float)cos(a), (float)sin(a));
    }
  }
  g_off_ready = true;
}
}  // namespace

// The tables live in a static device array (28 KB), so no call of the
// library allocates device memory for them. Every device holds its own copy;
// host code reaches it only through the address hipGetSymbolAddress returns
// (the array's name in host code is a host-side stand-in, not that address).
static __device__ __align__(256) float2 tw_table[kTwTotal];

hipError_t ensure_device_tables() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  build_offsets();
  if (g_tw[dev]) return hipSuccess;
  void *d = nullptr;
  e = hipGetSymbolAddress(&d, HIP_SYMBOL(tw_table));
  if (e != hipSuccess) return e;
  e = hipMemcpy(d, g_tw_host, sizeof(g_tw_host), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  g_tw[dev] = reinterpret_cast<float2 *>(d);
  return hipSuccess;
}

const float2 *twiddles(int n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  if (!g_tw[dev] || n < 1 || n > kMaxLen || g_tw_off[n] < 0) return nullptr;
  return g_tw[dev] + g_tw_off[n];
}

void release_device_tables() {
  // The tables are static device memory, held until the process ends; this
  // only forgets the addresses, so the next call uploads them again.
  std::lock_guard<std::mutex> lk(g_mu);
  for (int d = 0; d < kMaxDev; ++d) g_tw[d] = nullptr;
}

// ---------------------------------------------------------------------------
// Variant table and autotuner
// ---------------------------------------------------------------------------

namespace {
std::mutex g_var_mu;
int g_variant[kFftKinds][kMaxLen + 1];
bool g_tuned[kFftKinds][kMaxLen + 1];
bool g_var_ready = false;

void init_variants() {
  if (g_var_ready) return;
  for (int k = 0; k < kFftKinds; ++k)
    for (int n = 0; n <= kMaxLen; ++n) {
      g_variant[k][n] = 1;
      g_tuned[k][n] = false;
    }
  g_var_ready = true;
}
}  // namespace

int fft_variant(int kind, int len) {
  std::lock_guard<std::mutex> lk(g_var_mu);
  init_variants();
  if (kind < 0 || kind >= kFftKinds || len < 0 || len > kMaxLen) return 1;
  return g_variant[kind][len];
}

void fft_set_variant(int kind, int len, int v) {
  std::lock_guard<std::mutex> lk(g_var_mu);
  init_variants();
  if (kind < 0 || kind >= kFftKinds || len < 0 || len > kMaxLen || v < 0 || v >= kTileVariants)
    return;
  g_variant[kind][len] = v;
  g_tuned[kind][len] = true;
}

static bool fft_tuned(int kind, int len) {
  std::lock_guard<std::mutex> lk(g_var_mu);
  init_variants();
  return g_tuned[kind][len];
}

// One launch of axis kernel `kind` over a volume S x N x M with variant v.
// pitch: spectrum row pitch of the m and n kinds (0: M/2 + 1, the natural
// layout); the s kinds always use the natural layout.
static hipError_t launch_kind(int kind, int v, const float *rin, float *rout, float2 *spec, int S,
                              int N, int M, float scale, const int *done, hipStream_t st,
                              int pitch = 0) {
  const long Mh = M / 2 + 1;
  const long P = pitch > 0 ? pitch : Mh;
  switch (kind) {
    case kFftR2cM: return launch_r2c_m_v(rin, spec, (long)S * N, M, v, done, st, nullptr, nullptr, (int)(pitch > 0 ? pitch : 0));
    case kFftC2rM: return launch_c2r_m_v(spec, rout, (long)S * N, M, scale, v, done, st, nullptr, nullptr, (int)(pitch > 0 ? pitch : 0));
    case kFftFwdN: return launch_strided_v(spec, N, (long)S * P, P, (long)N * P, P, false, v, done, st, Mh);
    case kFftInvN: return launch_strided_v(spec, N, (long)S * P, P, (long)N * P, P, true, v, done, st, Mh);
    case kFftFwdS: return launch_strided_v(spec, S, (long)N * Mh, (long)N * Mh, 0, (long)N * Mh, false, v, done, st);
    case kFftInvS: return launch_strided_v(spec, S, (long)N * Mh, (long)N * Mh, 0, (long)N * Mh, true, v, done, st);
    default: return hipErrorInvalidValue;
  }
}

static int kind_len(int kind, int S, int N, int M) {
  return (kind <= kFftC2rM) ? M : (kind <= kFftInvN) ? N : S;
}

hipError_t fft_autotune(int S, int N, int M, int pitch, bool force, hipStream_t st) {
  hipError_t e = ensure_device_tables();
  if (e != hipSuccess) return e;
  const long Mh = M / 2 + 1;
  const long NT = (long)S * N * M, nspec = (long)S * N * (pitch > Mh ? pitch : Mh);
  // Successive timed launches work on different buffers, together larger
  // than the GPU's last-level cache, so the timings include the HBM traffic
  // each tile shape really causes.
  const size_t rbytes = ((sizeof(float) * NT + 255) / 256) * 256;
  const size_t sbytes = ((sizeof(float2) * nspec + 255) / 256) * 256;
  const size_t per = rbytes + sbytes;
  int nbuf = (int)(((size_t)640 << 20) / per) + 1;
  if (nbuf > 8) nbuf = 8;
  char *pool = nullptr;
  if ((e = hipMalloc(&pool, per * nbuf)) != hipSuccess) return e;
  auto real_of = [&](int r) { return reinterpret_cast<float *>(pool + per * (r % nbuf)); };
  auto spec_of = [&](int r) { return reinterpret_cast<float2 *>(pool + per * (r % nbuf) + rbytes); };
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  e = hipMemsetAsync(pool, 0, per * nbuf, st);
  int r = 0;
  for (int kind = 0; e == hipSuccess && kind < kFftKinds; ++kind) {
    const int len = kind_len(kind, S, N, M);
    if (len <= 1 || (!force && fft_tuned(kind, len))) continue;
    float best = 1e30f;
    int bv = 1;
    // Strided passes move T-column row segments: only tiles whose segments
    // fill whole 128-byte lines (T >= 16) are candidates when one exists.
    // Narrower segments fetch each line twice, which an isolated timing of
    // a cache-resident buffer does not show.
    const bool strided = kind >= kFftFwdN;
    int tmax = 1;
    for (int v = 0; v < kTileVariants; ++v)
      tmax = tile_lines(len, kTileElems[v]) > tmax ? tile_lines(len, kTileElems[v]) : tmax;
    const int tmin = strided ? (tmax < 16 ? tmax : 16) : 1;
    for (int v = 0; e == hipSuccess && v < kTileVariants; ++v) {
      if (tile_lines(len, kTileElems[v]) < tmin) continue;
      const int kp = (kind == kFftFwdS || kind == kFftInvS) ? 0 : pitch;
      e = launch_kind(kind, v, real_of(r), real_of(r), spec_of(r), S, N, M, 1.0f, nullptr, st, kp);
      ++r;
      if (e == hipSuccess) e = hipEventRecord(e0, st);
      for (int k = 0; e == hipSuccess && k < 5; ++k, ++r)
        e = launch_kind(kind, v, real_of(r), real_of(r), spec_of(r), S, N, M, 1.0f, nullptr, st,
                        kp);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && ms < best) {
        best = ms;
        bv = v;
      }
    }
    if (e == hipSuccess) fft_set_variant(kind, len, bv);
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(pool);
  return e;
}

int fft_tune_save(const char *path) {
  FILE *f = fopen(path, "w");
  if (!f) return -1;
  std::lock_guard<std::mutex> lk(g_var_mu);
  init_variants();
  fprintf(f, "# sr3d FFT tile choices: kind length variant (tile %d/%d/%d elements)\n",
          kTileElems[0], kTileElems[1], kTileElems[2]);
  for (int k = 0; k < kFftKinds; ++k)
    for (int n = 0; n <= kMaxLen; ++n)
      if (g_tuned[k][n]) fprintf(f, "%d %d %d\n", k, n, g_variant[k][n]);
  fclose(f);
  return 0;
}

int fft_tune_load(const char *path) {
  FILE *f = fopen(path, "r");
  if (!f) return -1;
  char line[256];
  int count = 0;
  while (fgets(line, sizeof line, f)) {
    int k, n, v;
    if (line[0] == '#') continue;
    if (sscanf(line, "%d %d %d", &k, &n, &v) == 3) {
      fft_set_variant(k, n, v);
      ++count;
    }
  }
  fclose(f);
  return count;
}

// ---------------------------------------------------------------------------
// 3D transforms
// ---------------------------------------------------------------------------

static hipError_t run_kind(int kind, int stage, const float *rin, float *rout, float2 *spec, int S,
                           int N, int M, float scale, const int *done, hipStream_t st) {
  const int len = kind_len(kind, S, N, M);
  if (kind >= kFftFwdN && len == 1) return hipSuccess;
  prof_begin(stage, st);
  hipError_t e = launch_kind(kind, fft_variant(kind, len), rin, rout, spec, S, N, M, scale, done, st);
  prof_end(st);
  return e;
}

hipError_t fft3d_forward(const float *in, float2 *spec, int S, int N, int M, const int *done,
                         hipStream_t st) {
  hipError_t e = run_kind(kFftR2cM, kStFftR2cM, in, nullptr, spec, S, N, M, 1.0f, done, st);
  if (e == hipSuccess) e = run_kind(kFftFwdN, kStFftN, nullptr, nullptr, spec, S, N, M, 1.0f, done, st);
  if (e == hipSuccess) e = run_kind(kFftFwdS, kStFftS, nullptr, nullptr, spec, S, N, M, 1.0f, done, st);
  return e;
}

hipError_t fft3d_forward_stack(const float *in, float2 *spec, int K, int S, int N, int M,
                               const int *done, hipStream_t st) {
  // m and n: the K volumes are K S planes of rows and columns; s: the columns
  // of every volume, each volume's lines starting S N Mh further.
  hipError_t e = run_kind(kFftR2cM, kStFftR2cM, in, nullptr, spec, K * S, N, M, 1.0f, done, st);
  if (e == hipSuccess) e = run_kind(kFftFwdN, kStFftN, nullptr, nullptr, spec, K * S, N, M, 1.0f, done, st);
  if (e == hipSuccess && S > 1) {
    const long Mh = M / 2 + 1;
    prof_begin(kStFftS, st);
    e = launch_strided_v(spec, S, (long)K * N * Mh, (long)N * Mh, (long)S * N * Mh, (long)N * Mh,
                         false, fft_variant(kFftFwdS, S), done, st);
    prof_end(st);
  }
  return e;
}

hipError_t fft3d_inverse(float2 *spec, float *out, int S, int N, int M, float scale,
                         const int *done, hipStream_t st) {
  hipError_t e = run_kind(kFftInvS, kStIfftS, nullptr, nullptr, spec, S, N, M, 1.0f, done, st);
  if (e == hipSuccess) e = run_kind(kFftInvN, kStIfftN, nullptr, nullptr, spec, S, N, M, 1.0f, done, st);
  if (e == hipSuccess) e = run_kind(kFftC2rM, kStIfftC2rM, nullptr, out, spec, S, N, M, scale, done, st);
  return e;
}

// n-axis pass over a spectrum with rows `pitch` apart (padding columns skipped).
static hipError_t run_n_pitched(bool inv, float2 *spec, int S, int N, int M, int pitch,
                                const int *done, hipStream_t st, const RedArgs *red = nullptr) {
  if (N == 1) return red ? hipErrorInvalidValue : hipSuccess;
  const int kind = inv ? kFftInvN : kFftFwdN;
  prof_begin(inv ? kStIfftN : kStFftN, st);
  const hipError_t e = launch_strided_v(spec, N, (long)S * pitch, pitch, (long)N * pitch, pitch,
                                        inv, fft_variant(kind, N), done, st, M / 2 + 1, red);
  prof_end(st);
  return e;
}

hipError_t fft_n_forward(float2 *spec, int S, int N, int M, int pitch, const int *done,
                         hipStream_t st, const RedArgs *red) {
  return run_n_pitched(false, spec, S, N, M, pitch, done, st, red);
}

hipError_t fft2d_mn_forward(const float *in, float2 *spec, int S, int N, int M, const int *kofp,
                            const int *posk, int pitch, const int *done, hipStream_t st,
                            const RedArgs *red) {
  prof_begin(kStFftR2cM, st);
  hipError_t e = launch_r2c_m_v(in, spec, (long)S * N, M, fft_variant(kFftR2cM, M), done, st,
                                kofp, posk, pitch, red);
  prof_end(st);
  if (e == hipSuccess) e = run_n_pitched(false, spec, S, N, M, pitch, done, st);
  return e;
}

hipError_t fft2d_mn_inverse(float2 *spec, float *out, int S, int N, int M, float scale,
                            const int *kofp, const int *posk, int pitch, const int *done,
                            hipStream_t st) {
  hipError_t e = run_n_pitched(true, spec, S, N, M, pitch, done, st);
  if (e == hipSuccess) {
    prof_begin(kStIfftC2rM, st);
    e = launch_c2r_m_v(spec, out, (long)S * N, M, scale, fft_variant(kFftC2rM, M), done, st,
                       kofp, posk, pitch);
    prof_end(st);
  }
  return e;
}

}  // namespace sr3d
