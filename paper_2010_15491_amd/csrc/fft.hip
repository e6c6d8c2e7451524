// 3D FFT for gfx950: Stockham autosort passes in LDS, one launch per axis.
//
// The paper needs one forward and one inverse 3D DFT per x-update (eq. (12)
// and Algorithm 1 step 5a). Volumes are [s][n][m] with m fastest:
//   * axis m: rows are contiguous; a workgroup loads T whole rows (coalesced),
//     transforms them in LDS and writes the half spectrum m/2+1 (R2C) or reads
//     the half spectrum and rebuilds the Hermitian row (C2R);
//   * axes n and s: lines are strided; a workgroup takes T adjacent columns
//     (the fastest index), so each element row it reads or writes is T
//     consecutive complex values (T*8 bytes), transforms in LDS, writes back
//     in place.
// In LDS element i of line t sits at lds[i*TP + t]; butterflies are mapped
// with t fastest across lanes, which keeps every pass conflict-free. Twiddles
// come from a per-device table computed once in FP64 and rounded to FP32,
// staged in LDS per workgroup. Inverse transforms use conj(DFT(conj(.))).
#include <math.h>
#include <mutex>
#include <vector>

#include "sr3d_internal.h"

namespace sr3d {

// ---------------------------------------------------------------------------
// Radix plan
// ---------------------------------------------------------------------------

struct Passes {
  int n;
  int r[16];
};

constexpr Passes make_passes(int N) {
  Passes P{0, {0}};
  int m = N;
  while (m % 3 == 0) { P.r[P.n++] = 3; m /= 3; }
  while (m % 8 == 0) { P.r[P.n++] = 8; m /= 8; }
  if (m % 4 == 0) { P.r[P.n++] = 4; m /= 4; }
  if (m % 2 == 0) { P.r[P.n++] = 2; m /= 2; }
  return P;
}

// Lines per workgroup: the largest power of two with T*N <= 8192, at most 64.
constexpr int tile_lines(int N) {
  int t = 1;
  while (t < 64 && 2 * t * N <= 8192) t *= 2;
  return t;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Forward DFT butterflies (sign -1).
template <int R> __device__ __forceinline__ void butterfly(float2 *v);

template <> __device__ __forceinline__ void butterfly<2>(float2 *v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void butterfly<3>(float2 *v) {
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 s = cadd(v[1], v[2]);
  float2 d = csub(v[1], v[2]);
  float2 t = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
  float2 e = make_float2(h * d.y, -h * d.x);  // -i h d
  v[0] = cadd(v[0], s);
  v[1] = cadd(t, e);
  v[2] = csub(t, e);
}

template <> __device__ __forceinline__ void butterfly<4>(float2 *v) {
  float2 t0 = cadd(v[0], v[2]);
  float2 t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]);
  float2 t3 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <> __device__ __forceinline__ void butterfly<8>(float2 *v) {
  const float c = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  butterfly<4>(e);
  butterfly<4>(o);
  // twiddles w8^k = exp(-i pi k / 4)
  float2 o1 = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
  float2 o2 = mul_mi(o[2]);
  float2 o3 = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

// One Stockham pass of radix R over T lines of length N in LDS. NS is the
// product of the radices of earlier passes. Reads all inputs into registers,
// barrier, writes outputs, barrier.
template <int N, int T, int TP, int R, int NS>
__device__ __forceinline__ void fft_pass(float2 *lds, const float2 *tw) {
  constexpr int NB = T * (N / R);
  constexpr int IPT = (NB + kThreads - 1) / kThreads;
  float2 v[IPT][R];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int w = threadIdx.x + it * kThreads;
    if ((NB % kThreads) == 0 || w < NB) {
      const int t = w % T, j = w / T;
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = lds[(j + r * (N / R)) * TP + t];
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[it][r] = cmul(v[it][r], tw[r * k * (N / (NS * R))]);
      }
      butterfly<R>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int w = threadIdx.x + it * kThreads;
    if ((NB % kThreads) == 0 || w < NB) {
      const int t = w % T, j = w / T;
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(base + r * NS) * TP + t] = v[it][r];
    }
  }
  __syncthreads();
}

template <int N, int T, int TP, int P, int NS>
__device__ __forceinline__ void fft_passes(float2 *lds, const float2 *tw) {
  constexpr Passes PL = make_passes(N);
  if constexpr (P < PL.n) {
    constexpr int R = PL.r[P];
    fft_pass<N, T, TP, R, NS>(lds, tw);
    fft_passes<N, T, TP, P + 1, NS * R>(lds, tw);
  }
}

template <int N>
__device__ __forceinline__ void stage_twiddles(float2 *stw, const float2 *__restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += kThreads) stw[i] = tw[i];
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Axis m, real -> half spectrum. nrows rows of N reals, output rows of N/2+1.
template <int N>
__global__ __launch_bounds__(kThreads) void k_fft_m_r2c(const float *__restrict__ in,
                                                        float2 *__restrict__ out, int nrows,
                                                        const float2 *__restrict__ tw,
                                                        const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(N), TP = T + 1, MH = N / 2 + 1;
  __shared__ float2 lds[N * TP];
  __shared__ float2 stw[N];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<N>(stw, tw);
  for (int w = threadIdx.x; w < N * T; w += kThreads) {
    const int i = w % N, t = w / N;
    const long r = row0 + t;
    const float v = (r < nrows) ? in[r * N + i] : 0.f;
    lds[i * TP + t] = make_float2(v, 0.f);
  }
  __syncthreads();
  fft_passes<N, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < MH * T; w += kThreads) {
    const int k = w % MH, t = w / MH;
    const long r = row0 + t;
    if (r < nrows) out[r * MH + k] = lds[k * TP + t];
  }
}

// Axis m, half spectrum -> real, times `scale`.
template <int N>
__global__ __launch_bounds__(kThreads) void k_fft_m_c2r(const float2 *__restrict__ in,
                                                        float *__restrict__ out, int nrows,
                                                        float scale,
                                                        const float2 *__restrict__ tw,
                                                        const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(N), TP = T + 1, MH = N / 2 + 1;
  __shared__ float2 lds[N * TP];
  __shared__ float2 stw[N];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<N>(stw, tw);
  for (int w = threadIdx.x; w < N * T; w += kThreads) {
    const int k = w % N, t = w / N;
    const long r = row0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (r < nrows) {
      // conj of the Hermitian-completed row: conj(X[k]) for stored k, and
      // conj(conj(X[N-k])) = X[N-k] for the mirrored half.
      if (k < MH) {
        v = in[r * MH + k];
        v.y = -v.y;
      } else {
        v = in[r * MH + (N - k)];
      }
    }
    lds[k * TP + t] = v;
  }
  __syncthreads();
  fft_passes<N, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < N * T; w += kThreads) {
    const int i = w % N, t = w / N;
    const long r = row0 + t;
    if (r < nrows) out[r * N + i] = lds[i * TP + t].x * scale;
  }
}

// Strided complex lines, in place. Column c (0 <= c < ncols) starts at
// (c / inner) * outer_stride + (c % inner); element i is at + i * estride.
template <int N, bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_strided(float2 *__restrict__ data, int ncols,
                                                          FastDiv inner, long outer_stride,
                                                          long estride,
                                                          const float2 *__restrict__ tw,
                                                          const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(N);
  __shared__ float2 lds[N * T];
  __shared__ float2 stw[N];
  const int t = threadIdx.x % T;  // fixed per thread since T divides kThreads
  const int c = blockIdx.x * T + t;
  const bool valid = c < ncols;
  long base = 0;
  if (valid) {
    const uint32_t q = inner.div((uint32_t)c);
    base = (long)q * outer_stride + (long)(c - q * inner.d);
  }
  stage_twiddles<N>(stw, tw);
  for (int w = threadIdx.x; w < N * T; w += kThreads) {
    const int i = w / T;
    float2 v = make_float2(0.f, 0.f);
    if (valid) {
      v = data[base + i * estride];
      if (INV) v.y = -v.y;
    }
    lds[i * T + t] = v;
  }
  __syncthreads();
  fft_passes<N, T, T, 0, 1>(lds, stw);
  if (valid) {
    for (int w = threadIdx.x; w < N * T; w += kThreads) {
      const int i = w / T;
      float2 v = lds[i * T + t];
      if (INV) v.y = -v.y;
      data[base + i * estride] = v;
    }
  }
}

// Length-1 axis m: copy with zero imaginary part / take real part.
__global__ void k_copy_r2c1(const float *in, float2 *out, long n, const int *done) {
  if (done && *done) return;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2(in[i], 0.f);
}
__global__ void k_copy_c2r1(const float2 *in, float *out, long n, float scale, const int *done) {
  if (done && *done) return;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i].x * scale;
}

// ---------------------------------------------------------------------------
// Twiddle tables (per device)
// ---------------------------------------------------------------------------

#define SR3D_FFT_LENGTHS(X) \
  X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
  X(384) X(512) X(768) X(1024)

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
std::mutex g_mu;
float2 *g_tw[kMaxDev] = {nullptr};
int g_tw_off[kMaxLen + 1];
bool g_off_ready = false;
size_t g_tw_total = 0;

void build_offsets() {
  if (g_off_ready) return;
  size_t off = 0;
  for (int n = 0; n <= kMaxLen; ++n) g_tw_off[n] = -1;
#define SR3D_OFF(L) g_tw_off[L] = (int)off; off += L;
  SR3D_FFT_LENGTHS(SR3D_OFF)
#undef SR3D_OFF
  g_tw_total = off;
  g_off_ready = true;
}
}  // namespace

hipError_t ensure_device_tables() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  build_offsets();
  if (g_tw[dev]) return hipSuccess;
  std::vector<float2> h(g_tw_total);
  for (int n = 1; n <= kMaxLen; ++n) {
    if (g_tw_off[n] < 0) continue;
    for (int k = 0; k < n; ++k) {
      const double a = -2.0 * M_PI * (double)k / (double)n;
      h[g_tw_off[n] + k] = make_float2((float)cos(a), (float)sin(a));
    }
  }
  float2 *d = nullptr;
  e = hipMalloc(&d, g_tw_total * sizeof(float2));
  if (e != hipSuccess) return e;
  e = hipMemcpy(d, h.data(), g_tw_total * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return e;
  }
  g_tw[dev] = d;
  return hipSuccess;
}

const float2 *twiddles(int n) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  if (!g_tw[dev] || n < 1 || n > kMaxLen || g_tw_off[n] < 0) return nullptr;
  return g_tw[dev] + g_tw_off[n];
}

void release_device_tables() {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < kMaxDev; ++d) {
    if (!g_tw[d]) continue;
    (void)hipSetDevice(d);
    (void)hipFree(g_tw[d]);
    g_tw[d] = nullptr;
  }
  (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static hipError_t launch_r2c_m_(const float *in, float2 *out, long nrows, int M, const int *done,
                                hipStream_t st) {
  if (M == 1) {
    const long n = nrows;
    hipLaunchKernelGGL(k_copy_r2c1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out,
                       n, done);
    return hipGetLastError();
  }
  const float2 *tw = twiddles(M);
  if (!tw) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_L(L)                                                                             \
  case L: {                                                                                   \
    constexpr int T = tile_lines(L);                                                          \
    hipLaunchKernelGGL(k_fft_m_r2c<L>, dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads), \
                       0, st, in, out, (int)nrows, tw, done);                                 \
    break;                                                                                    \
  }
    SR3D_FFT_LENGTHS(SR3D_L)
#undef SR3D_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_c2r_m_(const float2 *in, float *out, long nrows, int M, float scale,
                                const int *done, hipStream_t st) {
  if (M == 1) {
    const long n = nrows;
    hipLaunchKernelGGL(k_copy_c2r1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out,
                       n, scale, done);
    return hipGetLastError();
  }
  const float2 *tw = twiddles(M);
  if (!tw) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_L(L)                                                                             \
  case L: {                                                                                   \
    constexpr int T = tile_lines(L);                                                          \
    hipLaunchKernelGGL(k_fft_m_c2r<L>, dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads), \
                       0, st, in, out, (int)nrows, scale, tw, done);                          \
    break;                                                                                    \
  }
    SR3D_FFT_LENGTHS(SR3D_L)
#undef SR3D_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_strided_(float2 *data, int L, long ncols, long inner, long outer_stride,
                                  long estride, bool inv, const int *done, hipStream_t st) {
  if (L == 1) return hipSuccess;
  const float2 *tw = twiddles(L);
  if (!tw) return hipErrorInvalidValue;
  FastDiv fd((uint32_t)inner);
  switch (L) {
#define SR3D_L(LL)                                                                          \
  case LL: {                                                                                \
    constexpr int T = tile_lines(LL);                                                       \
    dim3 g((unsigned)((ncols + T - 1) / T));                                                \
    if (inv)                                                                                \
      hipLaunchKernelGGL((k_fft_strided<LL, true>), g, dim3(kThreads), 0, st, data,         \
                         (int)ncols, fd, outer_stride, estride, tw, done);                  \
    else                                                                                    \
      hipLaunchKernelGGL((k_fft_strided<LL, false>), g, dim3(kThreads), 0, st, data,        \
                         (int)ncols, fd, outer_stride, estride, tw, done);                  \
    break;                                                                                  \
  }
    SR3D_FFT_LENGTHS(SR3D_L)
#undef SR3D_L
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_r2c_m(const float *in, float2 *out, long nrows, int M, const int *done,
                               hipStream_t st) {
  prof_begin(kStFftR2cM, st);
  hipError_t e = launch_r2c_m_(in, out, nrows, M, done, st);
  prof_end(st);
  return e;
}

static hipError_t launch_c2r_m(const float2 *in, float *out, long nrows, int M, float scale,
                               const int *done, hipStream_t st) {
  prof_begin(kStIfftC2rM, st);
  hipError_t e = launch_c2r_m_(in, out, nrows, M, scale, done, st);
  prof_end(st);
  return e;
}

static hipError_t launch_strided(float2 *data, int L, long ncols, long inner, long outer_stride,
                                 long estride, bool inv, const int *done, hipStream_t st,
                                 int stage) {
  if (L == 1) return hipSuccess;
  prof_begin(stage, st);
  hipError_t e = launch_strided_(data, L, ncols, inner, outer_stride, estride, inv, done, st);
  prof_end(st);
  return e;
}

hipError_t fft3d_forward(const float *in, float2 *spec, int S, int N, int M, const int *done,
                         hipStream_t st) {
  const long Mh = M / 2 + 1;
  hipError_t e = launch_r2c_m(in, spec, (long)S * N, M, done, st);
  if (e != hipSuccess) return e;
  e = launch_strided(spec, N, (long)S * Mh, Mh, (long)N * Mh, Mh, false, done, st, kStFftN);
  if (e != hipSuccess) return e;
  return launch_strided(spec, S, (long)N * Mh, (long)N * Mh, 0, (long)N * Mh, false, done, st,
                        kStFftS);
}

hipError_t fft3d_inverse(float2 *spec, float *out, int S, int N, int M, float scale,
                         const int *done, hipStream_t st) {
  const long Mh = M / 2 + 1;
  hipError_t e = launch_strided(spec, S, (long)N * Mh, (long)N * Mh, 0, (long)N * Mh, true, done,
                                st, kStIfftS);
  if (e != hipSuccess) return e;
  e = launch_strided(spec, N, (long)S * Mh, Mh, (long)N * Mh, Mh, true, done, st, kStIfftN);
  if (e != hipSuccess) return e;
  return launch_c2r_m(spec, out, (long)S * N, M, scale, done, st);
}

}  // namespace sr3d
