// FFT along the strided axes n and s of a half spectrum, in place.
//
// Column c (0 <= c < ncols) of the launch starts at
// (c / inner) * outer_stride + (c % inner) and its element i lies i * estride
// further; columns with c % inner >= inner_valid are row padding and are
// neither read nor written. A workgroup takes T adjacent columns, so every element row it
// moves is T consecutive complex values; the lines are transformed in LDS
// (t fastest across lanes) and written back to the same places.
#include "fft_core.h"
#include "reduce.h"

namespace sr3d {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The same with two adjacent columns per thread, moved as 16-byte values:
// for rows of even length, even strides and a 16-byte aligned base, where
// columns 2i and 2i + 1 always lie side by side in one row.
template <int N, bool INV, int E>
__device__ __forceinline__ void strided_body_pairs(const StridedDesc &d, int bid, float2 *lds,
                                                   float2 *stw) {
  constexpr int T = tile_lines(N, E), TH = T / 2;
  const int tp = threadIdx.x % TH;  // fixed per thread since T / 2 divides kThreads
  const int c = bid * T + 2 * tp;
  bool v0 = c < d.ncols, v1 = false;
  long base = 0;
  if (v0) {
    const uint32_t q = d.inner.div((uint32_t)c);
    const int r = (int)(c - q * d.inner.d);
    v0 = r < d.inner_valid;
    v1 = r + 1 < d.inner_valid;
    base = (long)q * d.outer_stride + r;
  }
  f32x4 *data = reinterpret_cast<f32x4 *>(d.data);
  const long estride = d.estride / 2;
  constexpr int NT = N * TH;  // pairs in the tile
  constexpr int NE = (NT + kThreads - 1) / kThreads;
  const long b0 = v0 ? base / 2 : 0;
  f32x4 *l4 = reinterpret_cast<f32x4 *>(lds);
  {
    f32x4 v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      const int i = (NT % kThreads == 0 || w < NT) ? w / TH : 0;
      const f32x4 x = data[b0 + i * estride];
      v[k] = f32x4{v0 ? x.x : 0.f, v0 ? (INV ? -x.y : x.y) : 0.f, v1 ? x.z : 0.f,
                   v1 ? (INV ? -x.w : x.w) : 0.f};
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT) l4[w] = v[k];
    }
  }
  __syncthreads();
  fft_passes<N, T, T, 0, 1>(lds, stw);
  if (v0) {
    f32x4 v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT) v[k] = l4[w];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT) {
        const long e = b0 + (w / TH) * estride;
        const f32x4 o = f32x4{v[k].x, INV ? -v[k].y : v[k].y, v[k].z, INV ? -v[k].w : v[k].w};
        if (v1) data[e] = o;
        else reinterpret_cast<float2 *>(data)[2 * e] = make_float2(o.x, o.y);
      }
    }
  }
}

template <int N, bool INV, int E>
__device__ __forceinline__ void strided_body(const StridedDesc &d, int bid,
                                             const float2 *__restrict__ tw, float2 *lds,
                                             float2 *stw) {
  constexpr int T = tile_lines(N, E);
  if (((d.inner.d | d.outer_stride | d.estride) & 1) == 0 &&
      (reinterpret_cast<uintptr_t>(d.data) & 15) == 0) {
    stage_twiddles<N>(stw, tw);
    strided_body_pairs<N, INV, E>(d, bid, lds, stw);
    return;
  }
  const int t = threadIdx.x % T;  // fixed per thread since T divides kThreads
  const int c = bid * T + t;
  bool valid = c < d.ncols;
  long base = 0;
  if (valid) {
    const uint32_t q = d.inner.div((uint32_t)c);
    const int r = (int)(c - q * d.inner.d);
    valid = r < d.inner_valid;
    base = (long)q * d.outer_stride + r;
  }
  float2 *data = d.data;
  const long estride = d.estride;
  stage_twiddles<N>(stw, tw);
  // Element w of the tile (line t = w % T, the thread's own) sits at lds[w].
  // All of a thread's loads are issued before its first LDS store; a padding
  // or out-of-range column loads from column 0 and is zeroed.
  constexpr int NT = N * T;
  constexpr int NE = (NT + kThreads - 1) / kThreads;
  const long b0 = valid ? base : 0;
  {
    float2 v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      const int i = (NT % kThreads == 0 || w < NT) ? w / T : 0;
      const float2 x = data[b0 + i * estride];
      v[k] = valid ? make_float2(x.x, INV ? -x.y : x.y) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT) lds[w] = v[k];
    }
  }
  __syncthreads();
  fft_passes<N, T, T, 0, 1>(lds, stw);
  if (valid) {
    float2 v[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT) v[k] = lds[w];
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int w = threadIdx.x + k * kThreads;
      if (NT % kThreads == 0 || w < NT)
        data[base + (w / T) * estride] = make_float2(v[k].x, INV ? -v[k].y : v[k].y);
    }
  }
}

template <int N, bool INV, int E>
__global__ __launch_bounds__(kThreads) void k_fft_strided(StridedDesc d,
                                                          const float2 *__restrict__ tw) {
  // With a reduction attached, workgroup 0 (dispatched first, so it overlaps
  // the transform) runs the previous iteration's stopping test.
  const bool red = d.red.ctrl != nullptr;
  if (red && blockIdx.x == 0) {
    reduce_in_block(d.red);
    return;
  }
  if (d.done && *d.done) return;
  constexpr int T = tile_lines(N, E);
  __shared__ __align__(16) float2 lds[N * T];
  __shared__ float2 stw[N];
  strided_body<N, INV, E>(d, (int)blockIdx.x - (red ? 1 : 0), tw, lds, stw);
}

// Many volumes with the same line length: item (volume, tile) per workgroup.
template <int N, bool INV, int E>
__global__ __launch_bounds__(kThreads) void k_fft_strided_batch(const StridedDesc *__restrict__ descs,
                                                                const int2 *__restrict__ items,
                                                                const float2 *__restrict__ tw) {
  const int2 it = items[blockIdx.x];
  const StridedDesc d = descs[it.x];
  if (d.done && *d.done) return;
  constexpr int T = tile_lines(N, E);
  __shared__ __align__(16) float2 lds[N * T];
  __shared__ float2 stw[N];
  strided_body<N, INV, E>(d, it.y, tw, lds, stw);
}

template <int L, int E>
static void launch_strided_t(const StridedDesc &d, bool inv, hipStream_t st) {
  constexpr int T = tile_lines(L, E);
  dim3 g((unsigned)((d.ncols + T - 1) / T + (d.red.ctrl ? 1 : 0)));
  if (inv)
    hipLaunchKernelGGL((k_fft_strided<L, true, E>), g, dim3(kThreads), 0, st, d, twiddles(L));
  else
    hipLaunchKernelGGL((k_fft_strided<L, false, E>), g, dim3(kThreads), 0, st, d, twiddles(L));
}

template <int L, int E>
static void launch_strided_batch_t(const StridedDesc *descs, const int2 *items, int nitems, bool inv,
                                   hipStream_t st) {
  if (inv)
    hipLaunchKernelGGL((k_fft_strided_batch<L, true, E>), dim3(nitems), dim3(kThreads), 0, st,
                       descs, items, twiddles(L));
  else
    hipLaunchKernelGGL((k_fft_strided_batch<L, false, E>), dim3(nitems), dim3(kThreads), 0, st,
                       descs, items, twiddles(L));
}

int strided_tiles(int L, int v, long ncols) {
  int T = 1;
  switch (v) {
    case 0: T = 1; while (T < 64 && 2 * T * L <= kTileElems[0]) T *= 2; break;
    case 1: T = 1; while (T < 64 && 2 * T * L <= kTileElems[1]) T *= 2; break;
    default: T = 1; while (T < 64 && 2 * T * L <= kTileElems[2]) T *= 2; break;
  }
  return (int)((ncols + T - 1) / T);
}

hipError_t launch_strided_batch(int L, bool inv, int v, const StridedDesc *descs, const int2 *items,
                                int nitems, hipStream_t st) {
  if (L == 1 || nitems == 0) return hipSuccess;
  if (!twiddles(L)) return hipErrorInvalidValue;
  switch (L) {
#define SR3D_CASE(LL)                                                                     \
  case LL:                                                                                \
    if (v == 0) launch_strided_batch_t<LL, kTileElems[0]>(descs, items, nitems, inv, st); \
    else if (v == 1) launch_strided_batch_t<LL, kTileElems[1]>(descs, items, nitems, inv, st); \
    else launch_strided_batch_t<LL, kTileElems[2]>(descs, items, nitems, inv, st);        \
    break;
    SR3D_FFT_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_strided_v(float2 *data, int L, long ncols, long inner, long outer_stride,
                            long estride, bool inv, int v, const int *done, hipStream_t st,
                            long inner_valid, const RedArgs *red) {
  if (L == 1) return red ? hipErrorInvalidValue : hipSuccess;
  if (!twiddles(L)) return hipErrorInvalidValue;
  StridedDesc d = make_strided_desc(data, ncols, inner, outer_stride, estride, done, inner_valid);
  if (red) d.red = *red;
  switch (L) {
#define SR3D_CASE(LL)                                                           \
  case LL:                                                                      \
    if (v == 0) launch_strided_t<LL, kTileElems[0]>(d, inv, st);                \
    else if (v == 1) launch_strided_t<LL, kTileElems[1]>(d, inv, st);           \
    else launch_strided_t<LL, kTileElems[2]>(d, inv, st);                       \
    break;
    SR3D_FFT_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sr3d
