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
#include "reduce.h"

namespace sr3d {

template <int M, int E>
__device__ __forceinline__ void r2c_half_body(const RowDesc &d, int bid,
                                              const float2 *__restrict__ twh,
                                              const float2 *__restrict__ twm, float2 *lds,
                                              float2 *stw, int *sperm, float2 *stwm) {
  constexpr int H = M / 2, T = tile_lines(H, E), TP = T + 1, MH = M / 2 + 1;
  const long row0 = (long)bid * T;
  const long nrows = d.nrows;
  stage_twiddles<H>(stw, twh);
  for (int i = threadIdx.x; i < MH; i += kThreads) stwm[i] = twm[i];
  const bool perm = d.kofp != nullptr;
  const long pitch = d.pitch ? d.pitch : MH;
  if (perm)
    for (int i = threadIdx.x; i < MH; i += kThreads) sperm[i] = d.kofp[i];
  const float2 *in2 = reinterpret_cast<const float2 *>(d.rin);
  // all of a thread's loads are issued before its first LDS store
  constexpr int HT = H * T, NE = (HT + kThreads - 1) / kThreads;
  {
    float2 v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      const int i = w % H, t = w / H;
      const bool ok = (HT % kThreads == 0 || w < HT) && row0 + t < nrows;
      const float2 x = in2[(ok ? row0 + t : 0) * H + (ok ? i : 0)];
      v[k] = ok ? x : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (HT % kThreads == 0 || w < HT) lds[(w % H) * TP + w / H] = v[k];
    }
  }
  __syncthreads();
  fft_passes<H, T, TP, 0, 1>(lds, stw);
  float2 *out = d.spec;
  for (int w = threadIdx.x; w < MH * T; w += kThreads) {
    const int p = w % MH, t = w / MH;
    const long r = row0 + t;
    if (r < nrows) {
      const int k = perm ? sperm[p] : p;
      out[r * pitch + p] = r2c_post(lds[(k % H) * TP + t], lds[((H - k) % H) * TP + t], stwm[k]);
    }
  }
}

template <int M, int E>
__device__ __forceinline__ void c2r_half_body(const RowDesc &d, int bid,
                                              const float2 *__restrict__ twh,
                                              const float2 *__restrict__ twm, float2 *lds,
                                              float2 *stw, int *sperm, float2 *stwm) {
  constexpr int H = M / 2, T = tile_lines(H, E), TP = T + 1, MH = M / 2 + 1;
  const long row0 = (long)bid * T;
  const long nrows = d.nrows;
  const float2 *in = d.spec;
  stage_twiddles<H>(stw, twh);
  const bool perm = d.posk != nullptr;
  const long pitch = d.pitch ? d.pitch : MH;
  for (int i = threadIdx.x; i < H; i += kThreads) stwm[i] = twm[i];
  if (perm)
    for (int i = threadIdx.x; i < MH; i += kThreads) sperm[i] = d.posk[i];
  __syncthreads();
  // all of a thread's loads are issued before the first use
  constexpr int HT = H * T, NE = (HT + kThreads - 1) / kThreads;
  {
    float2 vk[NE], vm[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int w = threadIdx.x + q * kThreads;
      const int k = w % H, t = w / H;
      const bool ok = (HT % kThreads == 0 || w < HT) && row0 + t < nrows;
      const long rb = (ok ? row0 + t : 0) * pitch;
      vk[q] = in[rb + (perm ? sperm[k] : k)];
      vm[q] = in[rb + (perm ? sperm[H - k] : H - k)];
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const int w = threadIdx.x + q * kThreads;
      if (!(HT % kThreads == 0 || w < HT)) continue;
      const int k = w % H, t = w / H;
      float2 v = make_float2(0.f, 0.f);
      if (row0 + t < nrows) {
        const float2 xk = vk[q], xm = vm[q];
        // E = (X[k] + conj X[H-k]) / 2 ; O = e^{+2 pi i k/M} (X[k] - conj X[H-k]) / 2
        const float2 e = make_float2(0.5f * (xk.x + xm.x), 0.5f * (xk.y - xm.y));
        const float2 dd = make_float2(0.5f * (xk.x - xm.x), 0.5f * (xk.y + xm.y));
        const float2 wk = stwm[k];
        const float2 o = cmul(make_float2(wk.x, -wk.y), dd);
        // Z = E + i O, stored conjugated (inverse through the forward passes)
        v = make_float2(e.x - o.y, -(e.y + o.x));
      }
      lds[k * TP + t] = v;
    }
  }
  __syncthreads();
  fft_passes<H, T, TP, 0, 1>(lds, stw);
  // The unnormalised length-M inverse equals twice the length-M/2 one.
  const float s2 = 2.0f * d.scale;
  float2 *out2 = reinterpret_cast<float2 *>(d.rout);
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
__device__ __forceinline__ void r2c_full_body(const RowDesc &d, int bid,
                                              const float2 *__restrict__ tw, float2 *lds,
                                              float2 *stw) {
  constexpr int T = tile_lines(M, E), TP = T + 1, MH = M / 2 + 1;
  const long row0 = (long)bid * T;
  const long nrows = d.nrows;
  stage_twiddles<M>(stw, tw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int i = w % M, t = w / M;
    const long r = row0 + t;
    lds[i * TP + t] = make_float2((r < nrows) ? d.rin[r * M + i] : 0.f, 0.f);
  }
  __syncthreads();
  fft_passes<M, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < MH * T; w += kThreads) {
    const int k = w % MH, t = w / MH;
    const long r = row0 + t;
    if (r < nrows) d.spec[r * (d.pitch ? d.pitch : MH) + k] = lds[k * TP + t];
  }
}

template <int M, int E>
__device__ __forceinline__ void c2r_full_body(const RowDesc &d, int bid,
                                              const float2 *__restrict__ tw, float2 *lds,
                                              float2 *stw) {
  constexpr int T = tile_lines(M, E), TP = T + 1, MH = M / 2 + 1;
  const long row0 = (long)bid * T;
  const long nrows = d.nrows;
  stage_twiddles<M>(stw, tw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int k = w % M, t = w / M;
    const long r = row0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (r < nrows) {
      const long rp = r * (d.pitch ? d.pitch : MH);
      if (k < MH) {
        v = d.spec[rp + k];
        v.y = -v.y;
      } else {
        v = d.spec[rp + (M - k)];
      }
    }
    lds[k * TP + t] = v;
  }
  __syncthreads();
  fft_passes<M, T, TP, 0, 1>(lds, stw);
  for (int w = threadIdx.x; w < M * T; w += kThreads) {
    const int i = w % M, t = w / M;
    const long r = row0 + t;
    if (r < nrows) d.rout[r * M + i] = lds[i * TP + t].x * d.scale;
  }
}

// Kernels: single volume (blockIdx = row tile) and batch (item = volume, tile).
template <int M, int E, bool C2R>
__device__ __forceinline__ void row_body(const RowDesc &d, int bid, const float2 *twh,
                                         const float2 *twm) {
  if constexpr (M % 2 == 0) {
    constexpr int H = M / 2, T = tile_lines(H, E), TP = T + 1;
    __shared__ float2 lds[H * TP];
    __shared__ float2 stw[H];
    __shared__ int sperm[M / 2 + 1];
    __shared__ float2 stwm[M / 2 + 1];
    if (C2R) c2r_half_body<M, E>(d, bid, twh, twm, lds, stw, sperm, stwm);
    else r2c_half_body<M, E>(d, bid, twh, twm, lds, stw, sperm, stwm);
  } else {
    constexpr int T = tile_lines(M, E), TP = T + 1;
    __shared__ float2 lds[M * TP];
    __shared__ float2 stw[M];
    if (C2R) c2r_full_body<M, E>(d, bid, twm, lds, stw);
    else r2c_full_body<M, E>(d, bid, twm, lds, stw);
  }
}

template <int M, int E, bool C2R>
__global__ __launch_bounds__(kThreads) void k_fft_rows(RowDesc d, const float2 *__restrict__ twh,
                                                       const float2 *__restrict__ twm) {
  // With a reduction attached, workgroup 0 (dispatched first, so it overlaps
  // the transform) runs the previous iteration's stopping test.
  const bool red = !C2R && d.red.ctrl;
  if (red && blockIdx.x == 0) {
    reduce_in_block(d.red);
    return;
  }
  if (d.done && *d.done) return;
  row_body<M, E, C2R>(d, (int)blockIdx.x - (red ? 1 : 0), twh, twm);
}

template <int M, int E, bool C2R>
__global__ __launch_bounds__(kThreads) void k_fft_rows_batch(const RowDesc *__restrict__ descs,
                                                             const int2 *__restrict__ items,
                                                             const float2 *__restrict__ twh,
                                                             const float2 *__restrict__ twm) {
  const int2 it = items[blockIdx.x];
  const RowDesc d = descs[it.x];
  if (d.done && *d.done) return;
  row_body<M, E, C2R>(d, it.y, twh, twm);
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

constexpr int row_tile_lines(int M, int E) {
  return (M % 2 == 0) ? tile_lines(M / 2, E) : tile_lines(M, E);
}

template <int M, int E>
static void launch_rows_t(const RowDesc &d, bool c2r, hipStream_t st) {
  constexpr int T = row_tile_lines(M, E);
  const float2 *twh = (M % 2 == 0) ? twiddles(M / 2) : nullptr;
  dim3 g((unsigned)((d.nrows + T - 1) / T + (d.red.ctrl && !c2r ? 1 : 0)));
  if (c2r) hipLaunchKernelGGL((k_fft_rows<M, E, true>), g, dim3(kThreads), 0, st, d, twh, twiddles(M));
  else hipLaunchKernelGGL((k_fft_rows<M, E, false>), g, dim3(kThreads), 0, st, d, twh, twiddles(M));
}

template <int M, int E>
static void launch_rows_batch_t(const RowDesc *descs, const int2 *items, int nitems, bool c2r,
                                hipStream_t st) {
  const float2 *twh = (M % 2 == 0) ? twiddles(M / 2) : nullptr;
  if (c2r)
    hipLaunchKernelGGL((k_fft_rows_batch<M, E, true>), dim3(nitems), dim3(kThreads), 0, st, descs,
                       items, twh, twiddles(M));
  else
    hipLaunchKernelGGL((k_fft_rows_batch<M, E, false>), dim3(nitems), dim3(kThreads), 0, st, descs,
                       items, twh, twiddles(M));
}

int row_tiles(int M, int v, long nrows) {
  const int L = (M % 2 == 0) ? M / 2 : M;
  int T = 1;
  while (T < 64 && 2 * T * L <= kTileElems[v < 0 ? 0 : v > 2 ? 2 : v]) T *= 2;
  return (int)((nrows + T - 1) / T);
}

static hipError_t launch_rows(const RowDesc &d, int M, bool c2r, int v, hipStream_t st) {
  if (!twiddles(M) || (M % 2 == 0 && !twiddles(M / 2))) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_CASE(L)                                          \
  case L:                                                     \
    if (v == 0) launch_rows_t<L, kTileElems[0]>(d, c2r, st);  \
    else if (v == 1) launch_rows_t<L, kTileElems[1]>(d, c2r, st); \
    else launch_rows_t<L, kTileElems[2]>(d, c2r, st);         \
    break;
    SR3D_EVEN_M(SR3D_CASE)
    SR3D_CASE(3)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_batch(int M, bool c2r, int v, const RowDesc *descs, const int2 *items,
                             int nitems, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  if (M == 1 || !twiddles(M) || (M % 2 == 0 && !twiddles(M / 2))) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_CASE(L)                                                              \
  case L:                                                                         \
    if (v == 0) launch_rows_batch_t<L, kTileElems[0]>(descs, items, nitems, c2r, st); \
    else if (v == 1) launch_rows_batch_t<L, kTileElems[1]>(descs, items, nitems, c2r, st); \
    else launch_rows_batch_t<L, kTileElems[2]>(descs, items, nitems, c2r, st);    \
    break;
    SR3D_EVEN_M(SR3D_CASE)
    SR3D_CASE(3)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_r2c_m_v(const float *in, float2 *out, long nrows, int M, int v, const int *done,
                          hipStream_t st, const int *kofp, const int *posk, int pitch,
                          const RedArgs *red) {
  if (M == 1) {
    if (pitch > 1 || red) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_r2c1, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, in,
                       out, nrows, done);
    return hipGetLastError();
  }
  if (M % 2) kofp = posk = nullptr;  // odd M: every class order is the natural one
  RowDesc d{in, out, nullptr, nrows, 1.0f, done, kofp, posk, pitch, red ? *red : RedArgs{}};
  return launch_rows(d, M, false, v, st);
}

hipError_t launch_c2r_m_v(const float2 *in, float *out, long nrows, int M, float scale, int v,
                          const int *done, hipStream_t st, const int *kofp, const int *posk,
                          int pitch) {
  if (M == 1) {
    if (pitch > 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_c2r1, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, st, in,
                       out, nrows, scale, done);
    return hipGetLastError();
  }
  if (M % 2) kofp = posk = nullptr;
  RowDesc d{nullptr, const_cast<float2 *>(in), out, nrows, scale, done, kofp, posk, pitch, RedArgs{}};
  return launch_rows(d, M, true, v, st);
}

}  // namespace sr3d
