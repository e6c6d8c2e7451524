// Device core of the LDS Stockham FFT shared by the per-axis kernels.
#pragma once

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

// Lines per workgroup for a tile of at most E complex elements: the largest
// power of two with T*N <= E, at most 64.
constexpr int tile_lines(int N, int E) {
  int t = 1;
  while (t < 64 && 2 * t * N <= E) t *= 2;
  return t;
}

// Tile sizes (complex elements per workgroup) the autotuner chooses from.
constexpr int kTileVariants = 3;
constexpr int kTileElems[kTileVariants] = {2048, 4096, 8192};

// The FFT arithmetic below is never contracted into FMAs by the compiler:
// whether it would fuse a product into a later sum depends on the surrounding
// code (unrolling, tile shape), and every kernel that runs these transforms
// must produce the same bits for the same line. The fused multiply-adds it
// does use are explicit (fmaf), so they are the same in every kernel.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
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
#pragma clang fp contract(off)
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 s = cadd(v[1], v[2]);
  float2 d = csub(v[1], v[2]);
  float2 t = make_float2(fmaf(-0.5f, s.x, v[0].x), fmaf(-0.5f, s.y, v[0].y));
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
#pragma clang fp contract(off)
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

// Half-length real transform, last step: the length-M spectrum entry k from
// the length-M/2 complex spectrum Z of z[i] = x[2i] + i x[2i+1]:
//   X[k] = (Z[k] + conj Z[M/2-k]) / 2 - i e^{-2 pi i k/M} (Z[k] - conj Z[M/2-k]) / 2,
// with zk = Z[k mod M/2], zm = Z[(M/2-k) mod M/2] and wk = e^{-2 pi i k/M}.
// Every R2C kernel ends with this function.
__device__ __forceinline__ float2 r2c_post(float2 zk, float2 zm, float2 wk) {
#pragma clang fp contract(off)
  const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
  const float2 o = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
  // e + wk o
  return make_float2(fmaf(wk.x, o.x, fmaf(-wk.y, o.y, e.x)), fmaf(wk.x, o.y, fmaf(wk.y, o.x, e.y)));
}

template <int N>
__device__ __forceinline__ void stage_twiddles(float2 *stw, const float2 *__restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += kThreads) stw[i] = tw[i];
}


}  // namespace sr3d
