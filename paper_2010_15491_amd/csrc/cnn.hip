// Learned warm start: a 6-layer 3x3x3 CNN with 32 hidden channels applied to
// the Tikhonov solution, x0 = x + f(x), trained on the GPU.
//
// Layers: conv(1->32)+ReLU, 4 x conv(32->32)+ReLU, conv(32->1); periodic
// "same" padding; tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets along
// (s, n, m); conv(a)[v, co] = sum_t sum_ci W[t, co, ci] a[v + off_t, ci] + b[co].
// Weights and hidden activations are stored as bfloat16 (round to nearest
// even), activations channels-last ([voxel][32], 64 bytes); every sum is
// accumulated in FP32. Master parameters, gradients and Adam moments are FP32.
//
// The 32->32 layers (99% of the arithmetic) run on BF16 MFMA
// (v_mfma_f32_32x32x16_bf16) as implicit GEMMs: forward and input-gradient
// take 32-voxel x 32-channel output tiles, K = 27 taps x 32 channels, A rows
// gathered from an input plane staged in LDS, B from the layer's weights
// staged in LDS (k_conv32p below); the weight gradient contracts over
// voxels, with both operands staged transposed in LDS, one tap per
// wavefront, partial sums per workgroup reduced in a fixed order. The two
// single-channel layers run on the vector ALUs.
#include <stdint.h>

#include <type_traits>

#include "sr3d_internal.h"

namespace sr3d {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 32;
constexpr int NTAP = 27;
constexpr int W32 = NTAP * CH * CH;  // weights of a 32->32 layer
constexpr int W1 = NTAP * CH;        // weights of a 1->32 or 32->1 layer

// Parameter offsets (FP32 vector): per layer W (27, cout, cin) then b (cout).
constexpr long kOffW[6] = {0, W1 + CH, W1 + CH + (W32 + CH), W1 + CH + 2 * (W32 + CH),
                           W1 + CH + 3 * (W32 + CH), W1 + CH + 4 * (W32 + CH)};
constexpr long kCnnParams = kOffW[5] + W1 + 1;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct Vox {
  int s, n, m;
};

__device__ __forceinline__ Vox vox_of(long v, int N, int M) {
  Vox r;
  r.m = (int)(v % M);
  const long q = v / M;
  r.n = (int)(q % N);
  r.s = (int)(q / N);
  return r;
}

// neighbour index of (s, n, m) + sign * off_t, periodic
__device__ __forceinline__ long nbr(const Vox &p, int t, int sign, int S, int N, int M) {
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  int s = p.s + sign * dz, n = p.n + sign * dy, m = p.m + sign * dx;
  s = s < 0 ? s + S : (s >= S ? s - S : s);
  n = n < 0 ? n + N : (n >= N ? n - N : n);
  m = m < 0 ? m + M : (m >= M ? m - M : m);
  return ((long)s * N + n) * M + m;
}

// ---------------------------------------------------------------------------
// Parameter preparation, initialisation, Adam
// ---------------------------------------------------------------------------

// bf16 copy of all parameters (biases too, unused in bf16).
__global__ void k_params_bf16(const float *__restrict__ p, uint16_t *__restrict__ q, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = f2bf(p[i]);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)); the last layer is
// scaled by 0.1 so the initial warm start stays close to its input; biases 0.
__global__ void k_cnn_init(float *p, uint64_t seed) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kCnnParams) return;
  int l = 5;
  for (int k = 0; k < 6; ++k)
    if (i >= kOffW[k]) l = k;
  const int cin = l == 0 ? 1 : CH, cout = l == 5 ? 1 : CH;
  const long wn = (long)NTAP * cin * cout;
  const long r = i - kOffW[l];
  if (r >= wn) {
    p[i] = 0.f;
    return;
  }
  const double u = (double)(splitmix64(seed * 0x100000001B3ull + (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
  const double lim = sqrt(6.0 / (NTAP * cin)) * (l == 5 ? 0.1 : 1.0);
  p[i] = (float)((2.0 * u - 1.0) * lim);
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// 32 -> 32 layers on MFMA: forward (bias + ReLU) and input gradient (masked).
// ---------------------------------------------------------------------------

// A workgroup owns an 8 (n) x 32 (m) tile of output rows and a chunk of
// output planes along s. It streams the input planes of the chunk (plus one
// on each side) through LDS, one plane with its one-voxel n/m ring at a time,
// and every input plane is added into the three output planes it touches:
// output
// s = p - sg*dz takes tap dz of input plane p (sg = +1 forward, -1 for the
// input gradient, whose taps are mirrored). The three output planes in flight
// have their own accumulators, selected at compile time by the phase of p
// modulo 3, so each input voxel is read from HBM (1 + 2/8)(1 + 2/32) times per
// chunk instead of once per tap. Weights and the plane live in LDS with the
// 16-byte chunks of each 64-byte row XOR-swizzled by bits 2-3 of the row
// index: the LDS serves 16 lanes of a 16-byte read per cycle, and 16
// consecutive rows then cover its 64 banks once. Each
// wavefront computes two 32-voxel rows; per tap and channel half one weight
// operand serves both. The weights are MFMA's A operand and the voxels its B
// operand, so D is [co][voxel] and a lane stores four consecutive channels
// of one voxel at a time.
constexpr int kCvTN = 8;                   // n-rows per tile
constexpr int kCvHW = 34;                  // ring row width: 32 + 2
constexpr int kCvHalo = (kCvTN + 2) * kCvHW;
constexpr int kCvQ = kCvHalo * 4;          // 16-byte chunks of a ring plane
constexpr int kCvPf = (kCvQ + 255) / 256;  // chunks per thread

__device__ __forceinline__ int cv_swz(int row, int c) { return row * 64 + ((c ^ ((row >> 2) & 3)) << 4); }

struct Conv32Tile {
  int n0, m0, s0, s1;  // tile origin, output planes [s0, s1)
};

__device__ __forceinline__ Conv32Tile conv32_tile(int b, int S, int N, int M, int SC) {
  const int ntn = (N + kCvTN - 1) / kCvTN, ntm = (M + 31) / 32;
  const int t2 = b % (ntn * ntm), c = b / (ntn * ntm);
  Conv32Tile T;
  T.n0 = (t2 % ntn) * kCvTN;
  T.m0 = (t2 / ntn) * 32;
  T.s0 = c * SC;
  T.s1 = T.s0 + SC < S ? T.s0 + SC : S;
  return T;
}

// A thread's share of a ring plane (the tile's (8 + 2) x 34 voxels of one
// input plane, 64 bytes each, periodic): the offsets of its 16-byte chunks
// within an input plane and in LDS, and the chunks of the next plane in
// flight.
struct CvRing {
  int goff[kCvPf], loff[kCvPf];
  u32x4 pf[kCvPf];
  __device__ __forceinline__ void init(const Conv32Tile &T, int N, int M) {
#pragma unroll
    for (int k = 0; k < kCvPf; ++k) {
      const int q = threadIdx.x + k * 256;
      const int hv = q >> 2, c = q & 3, r = hv / kCvHW, col = hv - r * kCvHW;
      const int n = (T.n0 - 1 + r + N) % N, m = (T.m0 - 1 + col + M) % M;
      goff[k] = q < kCvQ ? (n * M + m) * 4 + c : -1;
      loff[k] = cv_swz(hv, c);
    }
  }
  __device__ __forceinline__ void fetch(const u32x4 *src, int p, int S, int N, int M) {
    const long pb = (long)((p + S) % S) * N * M * 4;
#pragma unroll
    for (int k = 0; k < kCvPf; ++k)
      if (goff[k] >= 0) pf[k] = src[pb + goff[k]];
  }
  __device__ __forceinline__ void put(char *pl) const {
#pragma unroll
    for (int k = 0; k < kCvPf; ++k)
      if (goff[k] >= 0) *reinterpret_cast<u32x4 *>(pl + loff[k]) = pf[k];
  }
};

template <bool DGRAD>
__global__ __launch_bounds__(256, 2) void k_conv32p(const uint16_t *__restrict__ in,
                                                    const uint16_t *__restrict__ wb,
                                                    const float *__restrict__ bias,
                                                    const uint16_t *__restrict__ mask, int S,
                                                    int N, int M, int SC,
                                                    uint16_t *__restrict__ out,
                                                    float *__restrict__ out_f32) {
  __shared__ __attribute__((aligned(16))) char wl[NTAP * CH * 64];  // [t][out] rows of 32 in
  __shared__ __attribute__((aligned(16))) char pl[kCvHalo * 64];    // one ring plane
  __shared__ float bl[CH];
  constexpr int sg = DGRAD ? -1 : 1;
  const Conv32Tile T = conv32_tile(blockIdx.x, S, N, M, SC);
  // Weights as 16-byte chunks: row t*32 + o holds in-channels c*8 .. c*8+7.
  for (int q = threadIdx.x; q < NTAP * CH * 4; q += 256) {
    const int row = q >> 2, c = q & 3, t = row >> 5, o = row & 31;
    u32x4 v;
    if (DGRAD) {  // out = ci, in = co: gather W[t][co][o] over co
      const uint16_t *w = wb + (long)t * CH * CH + c * 8 * CH + o;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = w[2 * j * CH] | ((uint32_t)w[(2 * j + 1) * CH] << 16);
    } else {
      v = *reinterpret_cast<const u32x4 *>(wb + (long)row * CH + c * 8);
    }
    *reinterpret_cast<u32x4 *>(wl + cv_swz(row, c)) = v;
  }
  if (threadIdx.x < CH) bl[threadIdx.x] = DGRAD ? 0.f : bias[threadIdx.x];
  CvRing ring;
  ring.init(T, N, M);
  const u32x4 *src = reinterpret_cast<const u32x4 *>(in);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kq = lane >> 5;
  f32x16 acc[3][2];
#pragma unroll
  for (int j = 0; j < 3; ++j) acc[j][0] = acc[j][1] = f32x16{};
  // Output rows of this wavefront: tile rows 2w and 2w + 1. D is [co][voxel]:
  // this lane holds channels g*8 + kq*4 .. + 3 (g = 0..3) of voxel m0 + col.
  auto emit = [&](int s, const f32x16 &a, int tt) __attribute__((always_inline)) {
    const int n = T.n0 + 2 * wave + tt, m = T.m0 + col;
    if (n >= N || m >= M) return;
    const long v = ((long)s * N + n) * M + m;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int co = g * 8 + kq * 4;
      float f[4];
      uint2 mk;
      if (DGRAD) mk = *reinterpret_cast<const uint2 *>(mask + v * CH + co);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float val = a[4 * g + e] + bl[co + e];
        if (DGRAD) {
          const uint32_t w = (e < 2 ? mk.x : mk.y) >> (16 * (e & 1));
          f[e] = bf2f((uint16_t)w) > 0.f ? val : 0.f;
        } else {
          f[e] = fmaxf(val, 0.f);
        }
      }
      *reinterpret_cast<uint2 *>(out + v * CH + co) =
          make_uint2(f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16), f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16));
      if (out_f32)
        *reinterpret_cast<float4 *>(out_f32 + v * CH + co) = make_float4(f[0], f[1], f[2], f[3]);
    }
  };
  // One input plane p at phase J = (p - s0 + 1) mod 3.
  auto step = [&](auto Jc, int p) __attribute__((always_inline)) {
    constexpr int J = decltype(Jc)::value;
    __syncthreads();  // every wavefront is done with the previous plane
    ring.put(pl);
    __syncthreads();
    if (p + 1 <= T.s1) ring.fetch(src, p + 1, S, N, M);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      const int so = p - sg * dz;
      if (so < T.s0 || so >= T.s1) continue;
      const int slot = ((J - sg * dz) % 3 + 3) % 3;
#pragma unroll 1
      for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int c = h * 2 + kq;
            const u32x4 bv = *reinterpret_cast<const u32x4 *>(wl + cv_swz(t * 32 + col, c));
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
              const int hv = (2 * wave + tt + 1 + sg * dy) * kCvHW + col + 1 + sg * dx;
              const u32x4 av = *reinterpret_cast<const u32x4 *>(pl + cv_swz(hv, c));
              f32x16 &A = slot == 0 ? acc[0][tt] : slot == 1 ? acc[1][tt] : acc[2][tt];
              A = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, bv),
                                                          __builtin_bit_cast(bf16x8, av), A, 0, 0, 0);
            }
          }
        }
      }
    }
    // Output plane p - 1 has now received all three input planes.
    const int so = p - 1;
    constexpr int done = (J + 2) % 3;
    if (so >= T.s0 && so < T.s1) {
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        emit(so, acc[done][tt], tt);
        acc[done][tt] = f32x16{};
      }
    }
  };
  ring.fetch(src, T.s0 - 1, S, N, M);
  for (int p = T.s0 - 1;; p += 3) {
    step(std::integral_constant<int, 0>{}, p);
    if (p + 1 > T.s1) break;
    step(std::integral_constant<int, 1>{}, p + 1);
    if (p + 2 > T.s1) break;
    step(std::integral_constant<int, 2>{}, p + 2);
    if (p + 3 > T.s1) break;
  }
}

// Layer 1 (1 -> 32) on MFMA, K = the 27 taps (padded to 32) of bf16(x). The
// same tiles and s-chunks as k_conv32p; the three input planes an output
// plane needs stay in LDS as bf16 rings (340 values each), and each plane is
// loaded once per chunk. D comes out as [co][voxel], so a lane holds four
// consecutive channels of one voxel per group and stores them as 8 bytes.
__global__ __launch_bounds__(256) void k_conv_in1(const float *__restrict__ x,
                                                  const uint16_t *__restrict__ wb,
                                                  const float *__restrict__ bias, int S, int N,
                                                  int M, int SC, uint16_t *__restrict__ out,
                                                  float *__restrict__ out_f32) {
  __shared__ uint16_t xl[3 * kCvHalo];
  const Conv32Tile T = conv32_tile(blockIdx.x, S, N, M, SC);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kq = lane >> 5;
  // A[co][tap] = W1[t][co]: this lane holds taps h*16 + kq*8 .. + 7 of channel col.
  u32x4 aw[2];
  // and, for the same taps, the ring offset (dy, dx) and the plane dz + 1 (3: padding)
  int toff[2][8], tdz[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int t = h * 16 + kq * 8 + j;
      const uint32_t w = t < NTAP ? wb[t * CH + col] : 0u;
      if (j & 1) aw[h][j >> 1] |= w << 16;
      else aw[h][j >> 1] = w;
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      toff[h][j] = (1 + dy) * kCvHW + col + 1 + dx;
      tdz[h][j] = t < NTAP ? dz + 1 : 3;
    }
  float bco[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) bco[r] = bias[(r / 4) * 8 + kq * 4 + (r % 4)];
  // ring plane q (periodic) -> slot (q - s0 + 1) mod 3; two values per thread
  float pf[2];
  int goff[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int hv = threadIdx.x + k * 256, r = hv / kCvHW, c = hv - r * kCvHW;
    goff[k] = hv < kCvHalo ? ((T.n0 - 1 + r + N) % N) * M + (T.m0 - 1 + c + M) % M : -1;
  }
  const long plane = (long)N * M;
  auto fetch = [&](int q) __attribute__((always_inline)) {
    const long pb = (long)((q + S) % S) * plane;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (goff[k] >= 0) pf[k] = x[pb + goff[k]];
  };
  auto put = [&](int slot) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (goff[k] >= 0) xl[slot * kCvHalo + threadIdx.x + k * 256] = f2bf(pf[k]);
  };
  fetch(T.s0 - 1);
  put(0);
  fetch(T.s0);
  put(1);
  if (T.s0 + 1 <= T.s1) fetch(T.s0 + 1);
  for (int s = T.s0; s < T.s1; ++s) {
    const int k0 = s - T.s0;
    put((k0 + 2) % 3);  // plane s + 1
    __syncthreads();
    if (s + 2 <= T.s1) fetch(s + 2);
    // LDS base of dz = -1, 0, 1
    const int b0 = (k0 % 3) * kCvHalo, b1 = ((k0 + 1) % 3) * kCvHalo, b2 = ((k0 + 2) % 3) * kCvHalo;
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int row = 2 * wave + tt;
      f32x16 acc = {};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        u32x4 bx;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int d = tdz[h][j];
          const int bs = d == 0 ? b0 : d == 1 ? b1 : b2;
          const uint32_t v = d < 3 ? xl[bs + row * kCvHW + toff[h][j]] : 0u;
          if (j & 1) bx[j >> 1] |= v << 16;
          else bx[j >> 1] = v;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, aw[h]),
                                                      __builtin_bit_cast(bf16x8, bx), acc, 0, 0, 0);
      }
      const int n = T.n0 + row, m = T.m0 + col;
      if (n < N && m < M) {
        const long v = ((long)s * N + n) * M + m;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float f[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) f[e] = fmaxf(acc[4 * g + e] + bco[4 * g + e], 0.f);
          const int co = g * 8 + kq * 4;
          *reinterpret_cast<uint2 *>(out + v * CH + co) =
              make_uint2(f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16),
                         f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16));
          if (out_f32)
            *reinterpret_cast<float4 *>(out_f32 + v * CH + co) = make_float4(f[0], f[1], f[2], f[3]);
        }
      }
    }
    __syncthreads();  // slot of plane s - 1 is free
  }
}

// Weight gradient of a 32 -> 32 layer: gW[t][co][ci] = sum_v g[v][co] a[v+off_t][ci],
// gb[co] = sum_v g[v][co]. Workgroups stride over 256-voxel chunks and write
// one partial (27*1024 + 32 floats) each.
constexpr int kWgChunk = 256;

__global__ __launch_bounds__(256) void k_conv32_wgrad(const uint16_t *__restrict__ a,
                                                      const uint16_t *__restrict__ g, int S,
                                                      int N, int M, float *__restrict__ partial) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[CH][kWgChunk];      // [co][v]
  __shared__ __attribute__((aligned(16))) uint16_t nT[4][CH][kWgChunk];   // per wave [ci][v]
  const long NV = (long)S * N * M;
  const long nchunks = (NV + kWgChunk - 1) / kWgChunk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kq = lane >> 5;
  f32x16 acc[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) acc[k] = f32x16{};
  float bsum = 0.f;
  for (long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const long c0 = ch * kWgChunk;
    __syncthreads();
    // g chunk, transposed (one voxel per thread); voxels past the end are zeros
    {
      const long v = c0 + threadIdx.x;
      uint4 d[4] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0),
                    make_uint4(0, 0, 0, 0)};
      if (v < NV) {
        const uint4 *row = reinterpret_cast<const uint4 *>(g + v * CH);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = row[q];
      }
      const uint16_t *e = reinterpret_cast<const uint16_t *>(d);
#pragma unroll
      for (int c = 0; c < CH; ++c) gT[c][threadIdx.x] = e[c];
    }
    __syncthreads();
    if (threadIdx.x < CH) {
      float s = 0.f;
      for (int vv = 0; vv < kWgChunk; ++vv) s += bf2f(gT[threadIdx.x][vv]);
      bsum += s;
    }
#pragma unroll
    for (int rd = 0; rd < 7; ++rd) {
      const int t = rd * 4 + wave;
      // each wave stages the shifted activations of its own tap (4 voxels per lane)
      if (t < NTAP) {
        for (int k = 0; k < kWgChunk / 64; ++k) {
          const int vv = lane + 64 * k;
          const long v = c0 + vv;
          uint4 d[4] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0),
                        make_uint4(0, 0, 0, 0)};
          if (v < NV) {
            const Vox p = vox_of(v, N, M);
            const uint4 *row = reinterpret_cast<const uint4 *>(a + nbr(p, t, 1, S, N, M) * CH);
#pragma unroll
            for (int q = 0; q < 4; ++q) d[q] = row[q];
          }
          const uint16_t *e = reinterpret_cast<const uint16_t *>(d);
#pragma unroll
          for (int c = 0; c < CH; ++c) nT[wave][c][vv] = e[c];
        }
      }
      __syncthreads();
      if (t < NTAP) {
        for (int kb = 0; kb < kWgChunk / 16; ++kb) {
          const uint4 av = *reinterpret_cast<const uint4 *>(&gT[col][kb * 16 + kq * 8]);
          const uint4 bv = *reinterpret_cast<const uint4 *>(&nT[wave][col][kb * 16 + kq * 8]);
          acc[rd] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                            __builtin_bit_cast(bf16x8, bv), acc[rd],
                                                            0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  float *pp = partial + (long)blockIdx.x * (W32 + CH);
#pragma unroll
  for (int rd = 0; rd < 7; ++rd) {
    const int t = rd * 4 + wave;
    if (t >= NTAP) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int co = (r / 4) * 8 + kq * 4 + (r % 4);
      pp[(long)t * CH * CH + co * CH + col] = acc[rd][r];
    }
  }
  if (threadIdx.x < CH) pp[W32 + threadIdx.x] = bsum;
}

// ---------------------------------------------------------------------------
// Layer 6 (32 -> 1): forward with residual and loss, and its backward.
// ---------------------------------------------------------------------------

// Plane-marching like k_conv32p, with one output channel: for each ring
// plane, MFMA forms Z[u][t] = sum_ci W6[t][ci] a[u][ci] for its 340 voxels
// and all 27 taps (B = W6 transposed, 27 of 32 columns used) into LDS, and
// the thread of output voxel v adds Z[v + off_t][t] over the 9 taps of each
// dz that reach its output planes in flight. Training also forms the loss
// gradient 2 (y - target) / NV and one partial sum of squares per workgroup.
constexpr int kCvZB = (kCvHalo + 31) / 32;  // 32-row blocks of a ring plane

__global__ __launch_bounds__(256, 2) void k_conv_out1(const uint16_t *__restrict__ a,
                                                      const uint16_t *__restrict__ wb,
                                                      const float *__restrict__ bias,
                                                      const float *__restrict__ x, int S, int N,
                                                      int M, int SC, float *__restrict__ y,
                                                      const float *__restrict__ target,
                                                      float *__restrict__ gout,
                                                      float *__restrict__ lpart) {
  __shared__ __attribute__((aligned(16))) char pl[kCvHalo * 64];
  __shared__ float zl[kCvHalo * NTAP];
  __shared__ float red[4];
  const Conv32Tile T = conv32_tile(blockIdx.x, S, N, M, SC);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kq = lane >> 5;
  // B[k = ci][n = t] = W6[t][ci]; this lane holds ci = h*16 + kq*8 .. + 7 of tap col.
  u32x4 bw[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ci = h * 16 + kq * 8 + 2 * j;
      bw[h][j] = col < NTAP ? (uint32_t)wb[col * CH + ci] | ((uint32_t)wb[col * CH + ci + 1] << 16)
                            : 0u;
    }
  CvRing ring;
  ring.init(T, N, M);
  const u32x4 *src = reinterpret_cast<const u32x4 *>(a);
  const float b0 = bias[0], inv_nv = 1.f / (float)((long)S * N * M);
  // output voxel of this thread: tile row r, column i
  const int r = threadIdx.x >> 5, i = threadIdx.x & 31;
  float acc[3] = {0.f, 0.f, 0.f}, r2 = 0.f;
  auto step = [&](auto Jc, int p) __attribute__((always_inline)) {
    constexpr int J = decltype(Jc)::value;
    __syncthreads();  // the previous plane's Z and ring are no longer read
    ring.put(pl);
    __syncthreads();
    if (p + 1 <= T.s1) ring.fetch(src, p + 1, S, N, M);
    for (int blk = wave; blk < kCvZB; blk += 4) {
      const int hv = blk * 32 + col;
      const int hc = hv < kCvHalo ? hv : kCvHalo - 1;
      f32x16 z = {};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const u32x4 av = *reinterpret_cast<const u32x4 *>(pl + cv_swz(hc, h * 2 + kq));
        z = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                    __builtin_bit_cast(bf16x8, bw[h]), z, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int hz = blk * 32 + (q / 4) * 8 + kq * 4 + (q % 4);
        if (hz < kCvHalo && col < NTAP) zl[hz * NTAP + col] = z[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      const int so = p - dz;
      if (so < T.s0 || so >= T.s1) continue;
      float sum = 0.f;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          sum += zl[((r + 1 + dy) * kCvHW + i + 1 + dx) * NTAP + t];
        }
      const int slot = ((J - dz) % 3 + 3) % 3;
      if (slot == 0) acc[0] += sum;
      else if (slot == 1) acc[1] += sum;
      else acc[2] += sum;
    }
    const int so = p - 1;
    constexpr int done = (J + 2) % 3;
    if (so >= T.s0 && so < T.s1) {
      const int n = T.n0 + r, m = T.m0 + i;
      if (n < N && m < M) {
        const long v = ((long)so * N + n) * M + m;
        const float yv = x[v] + (b0 + acc[done]);
        y[v] = yv;
        if (target) {
          const float d = yv - target[v];
          r2 += d * d;
          gout[v] = 2.f * d * inv_nv;
        }
      }
      acc[done] = 0.f;
    }
  };
  ring.fetch(src, T.s0 - 1, S, N, M);
  for (int p = T.s0 - 1;; p += 3) {
    step(std::integral_constant<int, 0>{}, p);
    if (p + 1 > T.s1) break;
    step(std::integral_constant<int, 1>{}, p + 1);
    if (p + 2 > T.s1) break;
    step(std::integral_constant<int, 2>{}, p + 2);
    if (p + 3 > T.s1) break;
  }
  if (target) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off);
    if (lane == 0) red[wave] = r2;
    __syncthreads();
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// g_a5[v][ci] = sum_t W6[t][ci] gout[v - off_t], masked by a5 > 0 -> bf16.
__global__ __launch_bounds__(256) void k_out1_dgrad(const float *__restrict__ gout,
                                                    const uint16_t *__restrict__ wb,
                                                    const uint16_t *__restrict__ a, int S, int N,
                                                    int M, uint16_t *__restrict__ gz,
                                                    float *__restrict__ gz_f32) {
  __shared__ float w[NTAP * CH];
  for (int i = threadIdx.x; i < NTAP * CH; i += 256) w[i] = bf2f(wb[i]);
  __syncthreads();
  const long NV = (long)S * N * M;
  const long v = (long)blockIdx.x * 256 + threadIdx.x;
  if (v >= NV) return;
  const Vox p = vox_of(v, N, M);
  float acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = 0.f;
  for (int t = 0; t < NTAP; ++t) {
    const float gv = gout[nbr(p, t, -1, S, N, M)];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] += w[t * CH + c] * gv;
  }
  for (int c = 0; c < CH; ++c) {
    const float val = bf2f(a[v * CH + c]) > 0.f ? acc[c] : 0.f;
    gz[v * CH + c] = f2bf(val);
    if (gz_f32) gz_f32[v * CH + c] = val;
  }
}

// Weight gradients of the single-channel layers, one partial per workgroup:
// OUT1=true : gW6[t][ci] = sum_v gout[v] a5[v+off_t][ci], gb6 = sum gout.
// OUT1=false: gW1[t][co] = sum_v g1[v][co] xb[v+off_t],   gb1[co] = sum_v g1[v][co].
constexpr int kSmallChunk = 512;

template <bool OUT1>
__global__ __launch_bounds__(256) void k_small_wgrad(const uint16_t *__restrict__ act,
                                                     const float *__restrict__ x,
                                                     const float *__restrict__ gout,
                                                     const uint16_t *__restrict__ g1, int S, int N,
                                                     int M, float *__restrict__ partial) {
  const long NV = (long)S * N * M;
  const long v0 = (long)blockIdx.x * kSmallChunk;
  // output o = t * 32 + c (864 of them) plus 32 (or 1) bias sums
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  for (long vv = 0; vv < kSmallChunk; ++vv) {
    const long v = v0 + vv;
    if (v >= NV) break;
    const Vox p = vox_of(v, N, M);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = threadIdx.x + k * 256;
      if (o >= NTAP * CH) continue;
      const int t = o / CH, c = o % CH;
      const long nb = nbr(p, t, 1, S, N, M);
      if (OUT1) acc[k] += gout[v] * bf2f(act[nb * CH + c]);
      else acc[k] += bf2f(g1[v * CH + c]) * bf2f(f2bf(x[nb]));
    }
    if (OUT1) {
      if (threadIdx.x == 0) bacc += gout[v];
    } else {
      if (threadIdx.x < CH) bacc += bf2f(g1[v * CH + threadIdx.x]);
    }
  }
  float *pp = partial + (long)blockIdx.x * (NTAP * CH + CH);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int o = threadIdx.x + k * 256;
    if (o < NTAP * CH) pp[o] = acc[k];
  }
  if (threadIdx.x < CH) pp[NTAP * CH + threadIdx.x] = bacc;
}

// out[i] = sum_b partial[b][i], fixed order.
__global__ void k_sum_partials(const float *__restrict__ partial, int nb, int stride, int n,
                               float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += partial[(long)b * stride + i];
  out[i] = s;
}

// loss = (sum of the per-workgroup squared residuals) / number of voxels
__global__ void k_sum_loss(const float *__restrict__ lpart, int nb, float inv_nv,
                           float *__restrict__ loss) {
  __shared__ float sh[16];
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += 1024) s += lpart[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < 16; ++w) t += sh[w];
    *loss = t * inv_nv;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

long cnn_param_count() { return kCnnParams; }
long cnn_w_offset(int l) { return kOffW[l]; }

static int wgrad_blocks(long NV) {
  const long ch = (NV + kWgChunk - 1) / kWgChunk;
  return (int)(ch < 512 ? ch : 512);
}
static int small_blocks(long NV) { return (int)((NV + kSmallChunk - 1) / kSmallChunk); }
// Grid of the plane-marching kernels: about 2048 workgroups (four rounds of
// two per CU), chunks of at least 4 output planes; returns the workgroups
// and sets the chunk length.
static int plane_grid(int S, int N, int M, int *SC) {
  const int t2 = ((N + kCvTN - 1) / kCvTN) * ((M + 31) / 32);
  int nsc = (2048 + t2 - 1) / t2;
  int sc = (S + nsc - 1) / nsc;
  sc = sc < 4 ? 4 : sc;
  sc = sc > S ? S : sc;
  *SC = sc;
  return t2 * ((S + sc - 1) / sc);
}

static void launch_conv32(bool dgrad, const uint16_t *in, const uint16_t *wb, const float *bias,
                          const uint16_t *mask, int S, int N, int M, uint16_t *out, float *out_f32,
                          hipStream_t st) {
  int SC;
  const dim3 grid((unsigned)plane_grid(S, N, M, &SC));
  if (dgrad)
    hipLaunchKernelGGL((k_conv32p<true>), grid, dim3(256), 0, st, in, wb, bias, mask, S, N, M, SC,
                       out, out_f32);
  else
    hipLaunchKernelGGL((k_conv32p<false>), grid, dim3(256), 0, st, in, wb, bias, mask, S, N, M, SC,
                       out, out_f32);
}

CnnWs cnn_layout(int S, int N, int M, bool training, char *base) {
  const long NV = (long)S * N * M;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  CnnWs L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += al(bytes);
    return p;
  };
  L.wbf = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * kCnnParams));
  const int nact = training ? 5 : 2;
  for (int i = 0; i < nact; ++i) L.act[i] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * NV * CH));
  if (training) {
    L.gz[0] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * NV * CH));
    L.gz[1] = reinterpret_cast<uint16_t *>(take(sizeof(uint16_t) * NV * CH));
    L.gout = reinterpret_cast<float *>(take(sizeof(float) * NV));
    L.y = reinterpret_cast<float *>(take(sizeof(float) * NV));
    const long pw = (long)wgrad_blocks(NV) * (W32 + CH);
    const long ps = (long)small_blocks(NV) * (NTAP * CH + CH);
    L.partial = reinterpret_cast<float *>(take(sizeof(float) * (pw > ps ? pw : ps)));
    int SC;
    L.lpart = reinterpret_cast<float *>(take(sizeof(float) * plane_grid(S, N, M, &SC)));
  }
  L.bytes = off + 256;
  return L;
}

hipError_t to_bf16(const float *p, uint16_t *q, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_params_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, q, n);
  return hipGetLastError();
}

hipError_t cnn_init(float *params, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_cnn_init, dim3((unsigned)((kCnnParams + 255) / 256)), dim3(256), 0, st,
                     params, seed);
  return hipGetLastError();
}

hipError_t cnn_adam(float *p, const float *g, float *m, float *v, int step, float lr, float b1,
                    float b2, float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((kCnnParams + 255) / 256)), dim3(256), 0, st, p, g,
                     m, v, (long)kCnnParams, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

// Forward through all layers. Training keeps every hidden activation
// (act[0..4]); inference ping-pongs two buffers. y = x + f(x).
hipError_t cnn_forward(int S, int N, int M, const float *params, const float *x, float *y,
                       const CnnWs &L, bool training, const float *target, float *gout,
                       float *lpart, hipStream_t st) {
  hipLaunchKernelGGL(k_params_bf16, dim3((unsigned)((kCnnParams + 255) / 256)), dim3(256), 0, st,
                     params, L.wbf, (long)kCnnParams);
  int SC;
  const int nb = plane_grid(S, N, M, &SC);
  hipLaunchKernelGGL(k_conv_in1, dim3(nb), dim3(256), 0, st, x, L.wbf + kOffW[0],
                     params + kOffW[0] + W1, S, N, M, SC, L.act[0], nullptr);
  for (int l = 1; l <= 4; ++l) {
    const uint16_t *in = training ? L.act[l - 1] : L.act[(l - 1) & 1];
    uint16_t *out = training ? L.act[l] : L.act[l & 1];
    launch_conv32(false, in, L.wbf + kOffW[l], params + kOffW[l] + W32, nullptr, S, N, M, out,
                  nullptr, st);
  }
  const uint16_t *a5 = training ? L.act[4] : L.act[0];
  hipLaunchKernelGGL(k_conv_out1, dim3(nb), dim3(256), 0, st, a5, L.wbf + kOffW[5],
                     params + kOffW[5] + W1, x, S, N, M, SC, y, target, gout, lpart);
  return hipGetLastError();
}

// Loss and full gradient (FP32) of the mean squared error against target.
hipError_t cnn_grad(int S, int N, int M, const float *params, const float *x, const float *target,
                    float *grad, float *loss, const CnnWs &L, hipStream_t st) {
  const long NV = (long)S * N * M;
  const unsigned vb = (unsigned)((NV + 255) / 256);
  hipError_t e = cnn_forward(S, N, M, params, x, L.y, L, true, target, L.gout, L.lpart, st);
  if (e != hipSuccess) return e;
  int SC;
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(1024), 0, st, L.lpart, plane_grid(S, N, M, &SC),
                     (float)(1.0 / (double)NV), loss);
  // layer 6
  const int sb = small_blocks(NV);
  hipLaunchKernelGGL((k_small_wgrad<true>), dim3(sb), dim3(256), 0, st, L.act[4], nullptr, L.gout,
                     nullptr, S, N, M, L.partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((NTAP * CH + 255) / 256), dim3(256), 0, st, L.partial,
                     sb, NTAP * CH + CH, NTAP * CH, grad + kOffW[5]);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, L.partial + NTAP * CH, sb,
                     NTAP * CH + CH, 1, grad + kOffW[5] + W1);
  hipLaunchKernelGGL(k_out1_dgrad, dim3(vb), dim3(256), 0, st, L.gout, L.wbf + kOffW[5], L.act[4],
                     S, N, M, L.gz[0], nullptr);
  // layers 5..2 (index l = 4..1): gz[cur] is the gradient at the layer output (pre-ReLU)
  int cur = 0;
  const int wb = wgrad_blocks(NV);
  for (int l = 4; l >= 1; --l) {
    hipLaunchKernelGGL(k_conv32_wgrad, dim3(wb), dim3(256), 0, st, L.act[l - 1], L.gz[cur], S, N,
                       M, L.partial);
    hipLaunchKernelGGL(k_sum_partials, dim3((W32 + CH + 255) / 256), dim3(256), 0, st, L.partial,
                       wb, W32 + CH, W32 + CH, grad + kOffW[l]);
    launch_conv32(true, L.gz[cur], L.wbf + kOffW[l], nullptr, L.act[l - 1], S, N, M, L.gz[cur ^ 1],
                  nullptr, st);
    cur ^= 1;
  }
  // layer 1
  hipLaunchKernelGGL((k_small_wgrad<false>), dim3(sb), dim3(256), 0, st, nullptr, x, nullptr,
                     L.gz[cur], S, N, M, L.partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((NTAP * CH + CH + 255) / 256), dim3(256), 0, st,
                     L.partial, sb, NTAP * CH + CH, NTAP * CH + CH, grad + kOffW[0]);
  return hipGetLastError();
}

// Single-layer primitives (building blocks, exposed for testing).
hipError_t conv_layer_forward(int S, int N, int M, int cin, int cout, const void *in,
                              const float *x, const uint16_t *wbf, const float *bias, void *out_bf16,
                              float *out_f32, hipStream_t st) {
  if (cin == 1 && cout == CH) {
    int SC;
    const int nb = plane_grid(S, N, M, &SC);
    hipLaunchKernelGGL(k_conv_in1, dim3(nb), dim3(256), 0, st, x, wbf, bias, S, N, M, SC,
                       (uint16_t *)out_bf16, out_f32);
  } else if (cin == CH && cout == CH) {
    launch_conv32(false, (const uint16_t *)in, wbf, bias, nullptr, S, N, M, (uint16_t *)out_bf16,
                  out_f32, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t conv_layer_backward(int S, int N, int M, const void *act_in, const void *gz,
                               const uint16_t *wbf, const void *mask, void *gin_bf16,
                               float *gin_f32, float *gw, float *partial, hipStream_t st) {
  const long NV = (long)S * N * M;
  const int wb = wgrad_blocks(NV);
  hipLaunchKernelGGL(k_conv32_wgrad, dim3(wb), dim3(256), 0, st, (const uint16_t *)act_in,
                     (const uint16_t *)gz, S, N, M, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((W32 + CH + 255) / 256), dim3(256), 0, st, partial, wb,
                     W32 + CH, W32 + CH, gw);
  if (gin_bf16)
    launch_conv32(true, (const uint16_t *)gz, wbf, nullptr, (const uint16_t *)mask, S, N, M,
                  (uint16_t *)gin_bf16, gin_f32, st);
  return hipGetLastError();
}

size_t conv_layer_partial_bytes(long NV) { return sizeof(float) * (size_t)wgrad_blocks(NV) * (W32 + CH); }

}  // namespace sr3d
