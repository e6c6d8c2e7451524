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
// take a 32-voxel x 32-channel output tile per wavefront, K = 27 taps x 32
// channels, A rows gathered from the neighbour voxels (16-byte loads), B from
// the layer's weights staged in LDS; the weight gradient contracts over
// voxels, with both operands staged transposed in LDS, one tap per
// wavefront, partial sums per workgroup reduced in a fixed order. The two
// single-channel layers run on the vector ALUs.
#include <stdint.h>

#include "sr3d_internal.h"

namespace sr3d {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

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
// Layer 1 (1 -> 32) on the vector ALUs.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_conv_in1(const float *__restrict__ x,
                                                  const uint16_t *__restrict__ wb,
                                                  const float *__restrict__ bias, int S, int N,
                                                  int M, uint16_t *__restrict__ out,
                                                  float *__restrict__ out_f32) {
  __shared__ float w[NTAP * CH], b[CH];
  for (int i = threadIdx.x; i < NTAP * CH; i += 256) w[i] = bf2f(wb[i]);
  if (threadIdx.x < CH) b[threadIdx.x] = bias[threadIdx.x];
  __syncthreads();
  const long NV = (long)S * N * M;
  const long v = (long)blockIdx.x * 256 + threadIdx.x;
  if (v >= NV) return;
  const Vox p = vox_of(v, N, M);
  float acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = b[c];
  for (int t = 0; t < NTAP; ++t) {
    const float xv = bf2f(f2bf(x[nbr(p, t, 1, S, N, M)]));
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] += w[t * CH + c] * xv;
  }
  uint32_t packed[CH / 2];
#pragma unroll
  for (int c = 0; c < CH; c += 2) {
    const float a0 = fmaxf(acc[c], 0.f), a1 = fmaxf(acc[c + 1], 0.f);
    packed[c / 2] = (uint32_t)f2bf(a0) | ((uint32_t)f2bf(a1) << 16);
    if (out_f32) {
      out_f32[v * CH + c] = a0;
      out_f32[v * CH + c + 1] = a1;
    }
  }
  uint4 *o = reinterpret_cast<uint4 *>(out + v * CH);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = make_uint4(packed[4 * k], packed[4 * k + 1], packed[4 * k + 2], packed[4 * k + 3]);
}

// ---------------------------------------------------------------------------
// 32 -> 32 layers on MFMA: forward (bias + ReLU) and input gradient (masked).
// ---------------------------------------------------------------------------

constexpr int kTilesPerWave = 4;  // 32-voxel tiles per wavefront

template <bool DGRAD>
__global__ __launch_bounds__(256) void k_conv32(const uint16_t *__restrict__ in,
                                                const uint16_t *__restrict__ wb,
                                                const float *__restrict__ bias,
                                                const uint16_t *__restrict__ mask, int S, int N,
                                                int M, uint16_t *__restrict__ out,
                                                float *__restrict__ out_f32) {
  // LDS weights as [t][out][in] with in contiguous: forward W[t][co][ci];
  // input gradient the transpose W[t][ci][co] (out = ci, in = co).
  __shared__ __attribute__((aligned(16))) uint16_t wl[W32];
  __shared__ float bl[CH];
  for (int i = threadIdx.x; i < W32; i += 256) {
    if (DGRAD) {
      const int t = i / (CH * CH), r = i % (CH * CH), o = r / CH, k = r % CH;
      wl[i] = wb[(long)t * CH * CH + k * CH + o];
    } else {
      wl[i] = wb[i];
    }
  }
  if (threadIdx.x < CH) bl[threadIdx.x] = DGRAD ? 0.f : bias[threadIdx.x];
  __syncthreads();
  const long NV = (long)S * N * M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kq = lane >> 5;
  for (int it = 0; it < kTilesPerWave; ++it) {
    const long tile = ((long)blockIdx.x * 4 + wave) * kTilesPerWave + it;
    const long v0 = tile * 32;
    if (v0 >= NV) break;
    long va = v0 + col;
    if (va >= NV) va = NV - 1;  // rows past the end compute junk, never stored
    const Vox p = vox_of(va, N, M);
    f32x16 acc = {};
    for (int t = 0; t < NTAP; ++t) {
      const long nb = nbr(p, t, DGRAD ? -1 : 1, S, N, M);
      const uint4 *arow = reinterpret_cast<const uint4 *>(in + nb * CH);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint4 av = arow[h * 2 + kq];
        const uint4 bv = *reinterpret_cast<const uint4 *>(&wl[(t * CH + col) * CH + h * 16 + kq * 8]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                      __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
      }
    }
    // D[row = voxel][col = output channel]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (r / 4) * 8 + kq * 4 + (r % 4);
      const long v = v0 + row;
      if (v < NV) {
        float val = acc[r] + bl[col];
        if (DGRAD) {
          if (!(bf2f(mask[v * CH + col]) > 0.f)) val = 0.f;
        } else {
          val = fmaxf(val, 0.f);
        }
        out[v * CH + col] = f2bf(val);
        if (out_f32) out_f32[v * CH + col] = val;
      }
    }
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

__global__ __launch_bounds__(256) void k_conv_out1(const uint16_t *__restrict__ a,
                                                   const uint16_t *__restrict__ wb,
                                                   const float *__restrict__ bias,
                                                   const float *__restrict__ x, int S, int N, int M,
                                                   float *__restrict__ y,
                                                   const float *__restrict__ target,
                                                   float *__restrict__ gout,
                                                   float *__restrict__ lpart) {
  __shared__ float w[NTAP * CH];
  __shared__ float red[4];
  for (int i = threadIdx.x; i < NTAP * CH; i += 256) w[i] = bf2f(wb[i]);
  __syncthreads();
  const long NV = (long)S * N * M;
  const long v = (long)blockIdx.x * 256 + threadIdx.x;
  float r2 = 0.f;
  if (v < NV) {
    const Vox p = vox_of(v, N, M);
    float acc = bias[0];
    for (int t = 0; t < NTAP; ++t) {
      const uint4 *row = reinterpret_cast<const uint4 *>(a + nbr(p, t, 1, S, N, M) * CH);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint4 d = row[q];
        const uint16_t *e = reinterpret_cast<const uint16_t *>(&d);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += w[t * CH + q * 8 + j] * bf2f(e[j]);
      }
    }
    const float yv = x[v] + acc;
    y[v] = yv;
    if (target) {
      const float r = yv - target[v];
      r2 = r * r;
      gout[v] = 2.f * r / (float)NV;
    }
  }
  if (target) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
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
static int conv32_blocks(long NV) {
  const long tiles = (NV + 31) / 32;
  return (int)((tiles + 4 * kTilesPerWave - 1) / (4 * kTilesPerWave));
}

CnnWs cnn_layout(long NV, bool training, char *base) {
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
    L.lpart = reinterpret_cast<float *>(take(sizeof(float) * ((NV + 255) / 256)));
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
  const long NV = (long)S * N * M;
  const unsigned vb = (unsigned)((NV + 255) / 256);
  hipLaunchKernelGGL(k_params_bf16, dim3((unsigned)((kCnnParams + 255) / 256)), dim3(256), 0, st,
                     params, L.wbf, (long)kCnnParams);
  hipLaunchKernelGGL(k_conv_in1, dim3(vb), dim3(256), 0, st, x, L.wbf + kOffW[0],
                     params + kOffW[0] + W1, S, N, M, L.act[0], nullptr);
  for (int l = 1; l <= 4; ++l) {
    const uint16_t *in = training ? L.act[l - 1] : L.act[(l - 1) & 1];
    uint16_t *out = training ? L.act[l] : L.act[l & 1];
    hipLaunchKernelGGL((k_conv32<false>), dim3(conv32_blocks(NV)), dim3(256), 0, st, in,
                       L.wbf + kOffW[l], params + kOffW[l] + W32, nullptr, S, N, M, out, nullptr);
  }
  const uint16_t *a5 = training ? L.act[4] : L.act[0];
  hipLaunchKernelGGL(k_conv_out1, dim3(vb), dim3(256), 0, st, a5, L.wbf + kOffW[5],
                     params + kOffW[5] + W1, x, S, N, M, y, target, gout, lpart);
  return hipGetLastError();
}

// Loss and full gradient (FP32) of the mean squared error against target.
hipError_t cnn_grad(int S, int N, int M, const float *params, const float *x, const float *target,
                    float *grad, float *loss, const CnnWs &L, hipStream_t st) {
  const long NV = (long)S * N * M;
  const unsigned vb = (unsigned)((NV + 255) / 256);
  hipError_t e = cnn_forward(S, N, M, params, x, L.y, L, true, target, L.gout, L.lpart, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(1024), 0, st, L.lpart, (int)vb,
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
    hipLaunchKernelGGL((k_conv32<true>), dim3(conv32_blocks(NV)), dim3(256), 0, st, L.gz[cur],
                       L.wbf + kOffW[l], nullptr, L.act[l - 1], S, N, M, L.gz[cur ^ 1], nullptr);
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
  const long NV = (long)S * N * M;
  const unsigned vb = (unsigned)((NV + 255) / 256);
  if (cin == 1 && cout == CH) {
    hipLaunchKernelGGL(k_conv_in1, dim3(vb), dim3(256), 0, st, x, wbf, bias, S, N, M,
                       (uint16_t *)out_bf16, out_f32);
  } else if (cin == CH && cout == CH) {
    hipLaunchKernelGGL((k_conv32<false>), dim3(conv32_blocks(NV)), dim3(256), 0, st,
                       (const uint16_t *)in, wbf, bias, nullptr, S, N, M, (uint16_t *)out_bf16,
                       out_f32);
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
    hipLaunchKernelGGL((k_conv32<true>), dim3(conv32_blocks(NV)), dim3(256), 0, st,
                       (const uint16_t *)gz, wbf, nullptr, (const uint16_t *)mask, S, N, M,
                       (uint16_t *)gin_bf16, gin_f32);
  return hipGetLastError();
}

size_t conv_layer_partial_bytes(long NV) { return sizeof(float) * (size_t)wgrad_blocks(NV) * (W32 + CH); }

}  // namespace sr3d
