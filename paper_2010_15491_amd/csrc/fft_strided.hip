// FFT along the strided axes n and s of a half spectrum, in place.
//
// Column c (0 <= c < ncols) of the launch starts at
// (c / inner) * outer_stride + (c % inner) and its element i lies i * estride
// further. A workgroup takes T adjacent columns, so every element row it
// moves is T consecutive complex values; the lines are transformed in LDS
// (t fastest across lanes) and written back to the same places.
#include "fft_core.h"

namespace sr3d {

template <int N, bool INV, int E>
__global__ __launch_bounds__(kThreads) void k_fft_strided(float2 *__restrict__ data, int ncols,
                                                          FastDiv inner, long outer_stride,
                                                          long estride,
                                                          const float2 *__restrict__ tw,
                                                          const int *__restrict__ done) {
  if (done && *done) return;
  constexpr int T = tile_lines(N, E);
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

template <int L, int E>
static void launch_strided_t(float2 *data, long ncols, FastDiv fd, long outer_stride, long estride,
                             bool inv, const int *done, hipStream_t st) {
  constexpr int T = tile_lines(L, E);
  dim3 g((unsigned)((ncols + T - 1) / T));
  if (inv)
    hipLaunchKernelGGL((k_fft_strided<L, true, E>), g, dim3(kThreads), 0, st, data, (int)ncols, fd,
                       outer_stride, estride, twiddles(L), done);
  else
    hipLaunchKernelGGL((k_fft_strided<L, false, E>), g, dim3(kThreads), 0, st, data, (int)ncols,
                       fd, outer_stride, estride, twiddles(L), done);
}

hipError_t launch_strided_v(float2 *data, int L, long ncols, long inner, long outer_stride,
                            long estride, bool inv, int v, const int *done, hipStream_t st) {
  if (L == 1) return hipSuccess;
  if (!twiddles(L)) return hipErrorInvalidValue;
  FastDiv fd((uint32_t)inner);
  switch (L) {
#define SR3D_CASE(LL)                                                                          \
  case LL:                                                                                     \
    if (v == 0) launch_strided_t<LL, kTileElems[0]>(data, ncols, fd, outer_stride, estride, inv, done, st); \
    else if (v == 1) launch_strided_t<LL, kTileElems[1]>(data, ncols, fd, outer_stride, estride, inv, done, st); \
    else launch_strided_t<LL, kTileElems[2]>(data, ncols, fd, outer_stride, estride, inv, done, st); \
    break;
    SR3D_FFT_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sr3d
