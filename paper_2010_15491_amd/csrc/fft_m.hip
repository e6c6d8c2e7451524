// FFT along the contiguous axis m: real rows <-> half-spectrum rows.
//
// Even lengths use the half-length method: a real row x of length M is read
// as M/2 complex values z[i] = x[2i] + i x[2i+1] (plain float2 loads), one
// complex FFT of length M/2 is done in LDS, and the half spectrum follows from
//   X[k] = (Z[k] + conj Z[M/2-k]) / 2 - i e^{-2 pi i k/M} (Z[k] - conj Z[M/2-k]) / 2
// for k = 0..M/2. The inverse undoes the same steps. Odd lengths (3) transform
// the real row as a complex one. A workgroup transforms T rows (T from the
// tile size the autotuner picked); rows are read and written coalesced.
#include "fft_core.h"

namespace sr3d {

template <int M, int E>
__global__ __launch_bounds__(kThreads) void k_r2c_half(const float *__restrict__ in,
                                                       float2 *__restrict__ out, int nrows,
                                                       const float2 *__restrict__ twh,
                                                       const float2 *__restrict__ twm,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int H = M / 2, T = tile_lines(H, E), TP = T + 1, MH = M / 2 + 1;
  __shared__ float2 lds[H * TP];
  __shared__ float2 stw[H];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<H>(stw, twh);
  const float2 *in2 = reinterpret_cast<const float2 *>(in);
  for (int w = threadIdx.x; w < H * T; w += kThreads) {
    const int i = w % H, t = w / H;
    const long r = row0 + t;
    lds[i * TP + t] = (r < nrows) ? in2[r * H + i] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_passes<H, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < MH * T; w += kThreads) {
    const int k = w % MH, t = w / MH;
    const long r = row0 + t;
    if (r < nrows) {
      const float2 zk = lds[(k % H) * TP + t];
      const float2 zm = lds[((H - k) % H) * TP + t];
      // E = (Z[k] + conj Z[H-k]) / 2 ; O = -i (Z[k] - conj Z[H-k]) / 2
      const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      const float2 wo = cmul(twm[k], o);
      out[r * MH + k] = make_float2(e.x + wo.x, e.y + wo.y);
    }
  }
}

template <int M, int E>
__global__ __launch_bounds__(kThreads) void k_c2r_half(const float2 *__restrict__ in,
                                                       float *__restrict__ out, int nrows,
                                                       float scale,
                                                       const float2 *__restrict__ twh,
                                                       const float2 *__restrict__ twm,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int H = M / 2, T = tile_lines(H, E), TP = T + 1, MH = M / 2 + 1;
  __shared__ float2 lds[H * TP];
  __shared__ float2 stw[H];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<H>(stw, twh);
  for (int w = threadIdx.x; w < H * T; w += kThreads) {
    const int k = w % H, t = w / H;
    const long r = row0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (r < nrows) {
      const float2 xk = in[r * MH + k];
      const float2 xm = in[r * MH + (H - k)];
      // E = (X[k] + conj X[H-k]) / 2 ; O = e^{+2 pi i k/M} (X[k] - conj X[H-k]) / 2
      const float2 e = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
      const float2 dd = make_float2(0.5f * (xk.x - xm.x), 0.5f * (xk.y + xm.y));
      const float2 wk = twm[k];
      const float2 o = cmul(make_float2(wk.x, -wk.y), dd);
      // Z = E + i O, stored conjugated (inverse through the forward passes)
      v = make_float2(e.x - o.y, -(e.y + o.x));
    }
    lds[k * TP + t] = v;
  }
  __syncthreads();
  fft_passes<H, T, TP, 0, 1>(lds, stw);
  // The unnormalised length-M inverse equals twice the length-M/2 one.
  const float s2 = 2.0f * scale;
  float2 *out2 = reinterpret_cast<float2 *>(out);
  for (int w = threadIdx.x; w < H * T; w += kThreads) {
    const int i = w % H, t = w / H;
    const long r = row0 + t;
    if (r < nrows) {
      const float2 v = lds[i * TP + t];
      out2[r * H + i] = make_float2(v.x * s2, -v.y * s2);
    }
  }
}

// Odd lengths: the real row transformed as a complex one.
template <int M, int E>
__global__ __launch_bounds__(kThreads) void k_r2c_full(const float *__restrict__ in,
                                                       float2 *__restrict__ out, int nrows,
                                                       const float2 *__restrict__ tw,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(M, E), TP = T + 1, MH = M / 2 + 1;
  __shared__ float2 lds[M * TP];
  __shared__ float2 stw[M];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<M>(stw, tw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int i = w % M, t = w / M;
    const long r = row0 + t;
    lds[i * TP + t] = make_float2((r < nrows) ? in[r * M + i] : 0.f, 0.f);
  }
  __syncthreads();
  fft_passes<M, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < MH * T; w += kThreads) {
    const int k = w % MH, t = w / MH;
    const long r = row0 + t;
    if (r < nrows) out[r * MH + k] = lds[k * TP + t];
  }
}

template <int M, int E>
__global__ __launch_bounds__(kThreads) void k_c2r_full(const float2 *__restrict__ in,
                                                       float *__restrict__ out, int nrows,
                                                       float scale,
                                                       const float2 *__restrict__ tw,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(M, E), TP = T + 1, MH = M / 2 + 1;
  __shared__ float2 lds[M * TP];
  __shared__ float2 stw[M];
  const long row0 = (long)blockIdx.x * T;
  stage_twiddles<M>(stw, tw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int k = w % M, t = w / M;
    const long r = row0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (r < nrows) {
      if (k < MH) {
        v = in[r * MH + k];
        v.y = -v.y;
      } else {
        v = in[r * MH + (M - k)];
      }
    }
    lds[k * TP + t] = v;
  }
  __syncthreads();
  fft_passes<M, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int i = w % M, t = w / M;
    const long r = row0 + t;
    if (r < nrows) out[r * M + i] = lds[i * TP + t].x * scale;
  }
}

// Length-1 axis m: copy with zero imaginary part / take the real part.
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

#define SR3D_EVEN_M(X)                                                                          \
  X(2) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) \
  X(512) X(768) X(1024)

template <int M, int E>
static void launch_r2c_t(const float *in, float2 *out, long nrows, const int *done,
                         hipStream_t st) {
  if constexpr (M % 2 == 0) {
    constexpr int T = tile_lines(M / 2, E);
    hipLaunchKernelGGL((k_r2c_half<M, E>), dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads),
                       0, st, in, out, (int)nrows, twiddles(M / 2), twiddles(M), done);
  } else {
    constexpr int T = tile_lines(M, E);
    hipLaunchKernelGGL((k_r2c_full<M, E>), dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads),
                       0, st, in, out, (int)nrows, twiddles(M), done);
  }
}

template <int M, int E>
static void launch_c2r_t(const float2 *in, float *out, long nrows, float scale, const int *done,
                         hipStream_t st) {
  if constexpr (M % 2 == 0) {
    constexpr int T = tile_lines(M / 2, E);
    hipLaunchKernelGGL((k_c2r_half<M, E>), dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads),
                       0, st, in, out, (int)nrows, scale, twiddles(M / 2), twiddles(M), done);
  } else {
    constexpr int T = tile_lines(M, E);
    hipLaunchKernelGGL((k_c2r_full<M, E>), dim3((unsigned)((nrows + T - 1) / T)), dim3(kThreads),
                       0, st, in, out, (int)nrows, scale, twiddles(M), done);
  }
}

hipError_t launch_r2c_m_v(const float *in, float2 *out, long nrows, int M, int v, const int *done,
                          hipStream_t st) {
  if (M == 1) {
    hipLaunchKernelGGL(k_copy_r2c1, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, in,
                       out, nrows, done);
    return hipGetLastError();
  }
  if (!twiddles(M)) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_CASE(L)                                                         \
  case L:                                                                    \
    if (v == 0) launch_r2c_t<L, kTileElems[0]>(in, out, nrows, done, st);    \
    else if (v == 1) launch_r2c_t<L, kTileElems[1]>(in, out, nrows, done, st); \
    else launch_r2c_t<L, kTileElems[2]>(in, out, nrows, done, st);           \
    break;
    SR3D_EVEN_M(SR3D_CASE)
    SR3D_CASE(3)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_c2r_m_v(const float2 *in, float *out, long nrows, int M, float scale, int v,
                          const int *done, hipStream_t st) {
  if (M == 1) {
    hipLaunchKernelGGL(k_copy_c2r1, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, in,
                       out, nrows, scale, done);
    return hipGetLastError();
  }
  if (!twiddles(M)) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_CASE(L)                                                                \
  case L:                                                                           \
    if (v == 0) launch_c2r_t<L, kTileElems[0]>(in, out, nrows, scale, done, st);    \
    else if (v == 1) launch_c2r_t<L, kTileElems[1]>(in, out, nrows, scale, done, st); \
    else launch_c2r_t<L, kTileElems[2]>(in, out, nrows, scale, done, st);           \
    break;
    SR3D_EVEN_M(SR3D_CASE)
    SR3D_CASE(3)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sr3d
