// l1 of orthonormal 3D Haar detail coefficients through the same x-step
// (Sec. III-B: other regularisers the ADMM splitting serves). With the split
// u = W x and W^T W = I, step 5a is the Tikhonov problem eq. (5) with
// 2 lambda -> mu and prior mean xbar = W^T (u - d), solved by the fold of
// eq. (12); steps 5b/5c act on wavelet coefficients:
//   nu = W x + d_prev, u' = soft(nu) on detail coefficients (identity on the
//   approximation ones), d' = nu - u', xbar' = W^T (u' - d').
// The state is nu (one plane, N_h floats). The coefficients are kept in place:
// level l transforms 2x2x2 blocks of the lattice of stride 2^(l-1), so the
// approximation coefficients of J levels sit at the multiples of 2^J.
#include "reduce.h"

// Exact rounding of every product and sum, as in the stencil kernels.
#pragma clang fp contract(off)
#include "stencil_core.h"

namespace sr3d {

// (a, b) -> ((a + b)/sqrt 2, (a - b)/sqrt 2) along each axis of a 2x2x2 block
// v[(a * 2 + b) * 2 + c] (a along s, b along n, c along m); the map is its own
// inverse, and applying it along m, n, s or s, n, m gives the same result in
// exact arithmetic; the forward and inverse passes use opposite orders.
__device__ __forceinline__ void haar_pairs(float *v, int stride) {
  const float h = 0.70710678118654752440f;
  for (int i = 0; i < 8; ++i) {
    if (i & stride) continue;
    const float e = v[i], o = v[i + stride];
    v[i] = (e + o) * h;
    v[i + stride] = (e - o) * h;
  }
}

// One level, in place: thread per 2x2x2 block of the stride-st lattice.
template <bool INV>
__global__ __launch_bounds__(kThreads) void k_haar_level(const float *__restrict__ in, float *out,
                                                         int S, int N, int M, int st,
                                                         const int *done) {
  if (done && *done) return;
  const int bm = M / (2 * st), bn = N / (2 * st), bs = S / (2 * st);
  const long b = (long)blockIdx.x * kThreads + threadIdx.x;
  if (b >= (long)bm * bn * bs) return;
  const int im = (int)(b % bm);
  const long r = b / bm;
  const int in_ = (int)(r % bn), is = (int)(r / bn);
  const long plane = (long)N * M;
  long off[8];
  float v[8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q = (a * 2 + bb) * 2 + c;
        off[q] = (long)(2 * is + a) * st * plane + (long)(2 * in_ + bb) * st * M + (long)(2 * im + c) * st;
        v[q] = in[off[q]];
      }
  if (INV) {
    haar_pairs(v, 4);  // s
    haar_pairs(v, 2);  // n
    haar_pairs(v, 1);  // m
  } else {
    haar_pairs(v, 1);
    haar_pairs(v, 2);
    haar_pairs(v, 4);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) out[off[q]] = v[q];
}

__device__ __forceinline__ float soft(float a, float thr) {
  return copysignf(fmaxf(fabsf(a) - thr, 0.f), a);
}

// Steps 5b/5c on the coefficients c = W x (in cz, overwritten by u' - d').
// mode 0: iteration (nu_in, stats); 1: start from c with d_prev = 0;
// 2: resume from nu_in alone (cz is only written).
template <typename Acc, int MODE>
__global__ __launch_bounds__(kThreads) void k_wavelet_admm(float *cz, const float *__restrict__ nu_in,
                                                           float *__restrict__ nu_out, int S, int N,
                                                           int M, int step, float thr, void *part,
                                                           const int *done) {
  if (done && *done) return;
  __shared__ Acc sh[6 * (kThreads / 64)];
  const long NT = (long)S * N * M;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (long v = (long)blockIdx.x * kThreads + threadIdx.x; v < NT; v += (long)gridDim.x * kThreads) {
    const int im = (int)(v % M);
    const long r = v / M;
    const int in_ = (int)(r % N), is = (int)(r / N);
    const bool detail = (im % step) | (in_ % step) | (is % step);
    const float t = detail ? thr : 0.f;
    if (MODE == 2) {
      const float nu = nu_in[v];
      const float u = soft(nu, t);
      cz[v] = u - (nu - u);
      continue;
    }
    const float c = cz[v];
    float dprev = 0.f, uold = 0.f;
    if (MODE == 0) {
      const float nuo = nu_in[v];
      uold = soft(nuo, t);
      dprev = nuo - uold;
    }
    const float nu = c + dprev;
    const float u = soft(nu, t);
    const float d = nu - u;
    nu_out[v] = nu;
    cz[v] = u - d;
    if (MODE == 0) {
      const float rp = c - u, du = u - uold;
      acc[0] += rp * rp;
      acc[1] += c * c;
      acc[2] += u * u;
      acc[3] += detail ? fabsf(c) : 0.f;
      acc[4] += du * du;
      acc[5] += d * d;
    }
  }
  if (MODE != 0) return;
  Acc acc_t[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) acc_t[q] = (Acc)acc[q];
  block_reduce_n<Acc>(acc_t, 6, sh);
  if (threadIdx.x == 0) {
    Acc *p = reinterpret_cast<Acc *>(part);
    for (int q = 0; q < 6; ++q) p[(long)q * gridDim.x + blockIdx.x] = acc_t[q];
  }
}

// All of steps 5b/5c with W and W^T for J <= 3 levels in one pass: a
// workgroup takes tiles of 2^J (s) x 2^J (n) x up to 64 (m) voxels (whole
// 2^J-cubes, which W maps onto themselves), transforms x in LDS, applies the
// shrink and dual update with nu read and written in row order, transforms
// back and stores xbar. Modes as k_wavelet_admm: 0 iteration, 1 start from x
// (x null: zero), 2 resume from nu_in.
constexpr int kWavTM = 64;

template <int J>
__device__ __forceinline__ void tile_levels(float *t, int tmv, bool inverse) {
  constexpr int T = 1 << J;
  for (int k = 0; k < J; ++k) {
    const int lev = inverse ? J - 1 - k : k;
    const int st = 1 << lev;
    const int bs = T / (2 * st), bm = tmv / (2 * st);
    const int nblk = bs * bs * bm;
    for (int q = threadIdx.x; q < nblk; q += kThreads) {
      const int ic = q % bm, r = q / bm, ib = r % bs, ia = r / bs;
      const int base = ((2 * ia * st) * T + 2 * ib * st) * kWavTM + 2 * ic * st;
      float v[8];
      int o[8];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int qq = (a * 2 + b2) * 2 + c;
            o[qq] = base + (a * st * T + b2 * st) * kWavTM + c * st;
            v[qq] = t[o[qq]];
          }
      if (inverse) {
        haar_pairs(v, 4);
        haar_pairs(v, 2);
        haar_pairs(v, 1);
      } else {
        haar_pairs(v, 1);
        haar_pairs(v, 2);
        haar_pairs(v, 4);
      }
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) t[o[qq]] = v[qq];
    }
    __syncthreads();
  }
}

template <typename Acc, int J, int MODE>
__global__ __launch_bounds__(kThreads) void k_wavelet_fused(const float *__restrict__ x,
                                                            const float *__restrict__ nu_in,
                                                            float *__restrict__ nu_out,
                                                            float *__restrict__ xbar, int S, int N,
                                                            int M, float thr, void *part,
                                                            const int *done) {
  constexpr int T = 1 << J, TE = T * T * kWavTM;
  if (done && *done) return;
  __shared__ float t[TE];
  __shared__ Acc sh[6 * (kThreads / 64)];
  const int tm = (M + kWavTM - 1) / kWavTM, tn = N / T, ts = S / T;
  const long ntiles = (long)ts * tn * tm;
  const long plane = (long)N * M;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int im = (int)(tile % tm);
    const long r = tile / tm;
    const int in_ = (int)(r % tn), is = (int)(r / tn);
    const int m0 = im * kWavTM, tmv = min(kWavTM, M - m0);
    const long g0 = (long)is * T * plane + (long)in_ * T * M + m0;
    // element e of the tile: row e / kWavTM = a T + b (s offset a, n offset b), m offset e % kWavTM
    auto gidx = [&](int e) {
      const int row = e / kWavTM, m = e % kWavTM;
      return g0 + (long)(row / T) * plane + (long)(row % T) * M + m;
    };
    if (MODE != 2) {
      for (int e = threadIdx.x; e < TE; e += kThreads)
        if (e % kWavTM < tmv) t[e] = x ? x[gidx(e)] : 0.f;
      __syncthreads();
      tile_levels<J>(t, tmv, false);
    }
    for (int e = threadIdx.x; e < TE; e += kThreads) {
      const int m = e % kWavTM;
      if (m >= tmv) continue;
      const int row = e / kWavTM;
      // approximation coefficients: multiples of 2^J along every axis, i.e.
      // the tile's first row and every 2^J-th m
      const bool detail = row != 0 || (m % T) != 0;
      const float th = detail ? thr : 0.f;
      const long gi = gidx(e);
      // The state nu is streamed (non-temporal): read and written once per
      // iteration, it would only displace x, xbar and the spectrum from the
      // last-level cache.
      if (MODE == 2) {
        const float nu = __builtin_nontemporal_load(nu_in + gi);
        const float u = soft(nu, th);
        t[e] = u - (nu - u);
        continue;
      }
      const float c = t[e];
      float dprev = 0.f, uold = 0.f;
      if (MODE == 0) {
        const float nuo = __builtin_nontemporal_load(nu_in + gi);
        uold = soft(nuo, th);
        dprev = nuo - uold;
      }
      const float nu = c + dprev;
      const float u = soft(nu, th);
      const float d = nu - u;
      __builtin_nontemporal_store(nu, nu_out + gi);
      t[e] = u - d;
      if (MODE == 0) {
        const float rp = c - u, du = u - uold;
        acc[0] += rp * rp;
        acc[1] += c * c;
        acc[2] += u * u;
        acc[3] += detail ? fabsf(c) : 0.f;
        acc[4] += du * du;
        acc[5] += d * d;
      }
    }
    __syncthreads();
    tile_levels<J>(t, tmv, true);
    for (int e = threadIdx.x; e < TE; e += kThreads)
      if (e % kWavTM < tmv) xbar[gidx(e)] = t[e];
    __syncthreads();  // the tile buffer is reloaded for the next tile
  }
  if (MODE != 0) return;
  Acc acc_t[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) acc_t[q] = (Acc)acc[q];
  block_reduce_n<Acc>(acc_t, 6, sh);
  if (threadIdx.x == 0) {
    Acc *p = reinterpret_cast<Acc *>(part);
    for (int q = 0; q < 6; ++q) p[(long)q * gridDim.x + blockIdx.x] = acc_t[q];
  }
}

int wavelet_fused_blocks(int S, int N, int M, int levels) {
  const int T = 1 << levels;
  const long tiles = (long)(S / T) * (N / T) * ((M + kWavTM - 1) / kWavTM);
  return (int)(tiles < 2048 ? (tiles < 1 ? 1 : tiles) : 2048);
}

template <int J>
static void launch_wf(const float *x, const float *nu_in, float *nu_out, float *xbar, int S, int N,
                      int M, float thr, int mode, void *part, bool fp64, const int *done,
                      hipStream_t st) {
  const dim3 g((unsigned)wavelet_fused_blocks(S, N, M, J)), b(kThreads);
  if (mode == 1)
    hipLaunchKernelGGL((k_wavelet_fused<float, J, 1>), g, b, 0, st, x, nu_in, nu_out, xbar, S, N,
                       M, thr, part, done);
  else if (mode == 2)
    hipLaunchKernelGGL((k_wavelet_fused<float, J, 2>), g, b, 0, st, x, nu_in, nu_out, xbar, S, N,
                       M, thr, part, done);
  else if (fp64)
    hipLaunchKernelGGL((k_wavelet_fused<double, J, 0>), g, b, 0, st, x, nu_in, nu_out, xbar, S, N,
                       M, thr, part, done);
  else
    hipLaunchKernelGGL((k_wavelet_fused<float, J, 0>), g, b, 0, st, x, nu_in, nu_out, xbar, S, N,
                       M, thr, part, done);
}

hipError_t wavelet_fused(const float *x, const float *nu_in, float *nu_out, float *xbar, int S,
                         int N, int M, int levels, float thr, int mode, void *part, bool fp64,
                         const int *done, hipStream_t st) {
  switch (levels) {
    case 1: launch_wf<1>(x, nu_in, nu_out, xbar, S, N, M, thr, mode, part, fp64, done, st); break;
    case 2: launch_wf<2>(x, nu_in, nu_out, xbar, S, N, M, thr, mode, part, fp64, done, st); break;
    case 3: launch_wf<3>(x, nu_in, nu_out, xbar, S, N, M, thr, mode, part, fp64, done, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int wavelet_blocks(int S, int N, int M) {
  const long NT = (long)S * N * M;
  long b = (NT + 8L * kThreads - 1) / (8L * kThreads);  // 8 voxels per thread
  if (b > 2048) b = 2048;
  return (int)(b < 1 ? 1 : b);
}

hipError_t haar3(const float *in, float *out, int S, int N, int M, int levels, bool inverse,
                 const int *done, hipStream_t st) {
  for (int k = 0; k < levels; ++k) {
    const int lev = inverse ? levels - 1 - k : k;
    const int s = 1 << lev;
    const long nb = (long)(S / (2 * s)) * (N / (2 * s)) * (M / (2 * s));
    // level 1 forward reads x and writes the coefficient buffer; the other
    // passes work in place on `out`
    const float *src = (!inverse && lev == 0) ? in : out;
    const dim3 g((unsigned)((nb + kThreads - 1) / kThreads));
    if (inverse)
      hipLaunchKernelGGL(k_haar_level<true>, g, dim3(kThreads), 0, st, src, out, S, N, M, s, done);
    else
      hipLaunchKernelGGL(k_haar_level<false>, g, dim3(kThreads), 0, st, src, out, S, N, M, s,
                         done);
    const hipError_t e = hipGetLastError();
    if (e) return e;
  }
  return hipSuccess;
}

hipError_t wavelet_admm(float *cz, const float *nu_in, float *nu_out, int S, int N, int M,
                        int levels, float thr, int mode, void *part, bool fp64, const int *done,
                        hipStream_t st) {
  const dim3 g((unsigned)wavelet_blocks(S, N, M)), b(kThreads);
  const int step = 1 << levels;
  if (mode == 1)
    hipLaunchKernelGGL((k_wavelet_admm<float, 1>), g, b, 0, st, cz, nu_in, nu_out, S, N, M, step,
                       thr, part, done);
  else if (mode == 2)
    hipLaunchKernelGGL((k_wavelet_admm<float, 2>), g, b, 0, st, cz, nu_in, nu_out, S, N, M, step,
                       thr, part, done);
  else if (fp64)
    hipLaunchKernelGGL((k_wavelet_admm<double, 0>), g, b, 0, st, cz, nu_in, nu_out, S, N, M, step,
                       thr, part, done);
  else
    hipLaunchKernelGGL((k_wavelet_admm<float, 0>), g, b, 0, st, cz, nu_in, nu_out, S, N, M, step,
                       thr, part, done);
  return hipGetLastError();
}

}  // namespace sr3d
