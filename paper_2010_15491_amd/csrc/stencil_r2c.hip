// The ADMM stencil (Algorithm 1 steps 5b, 5c and the Theta = L^T (u - d) of
// the next step 5a) with the next x-update's first transform fused in: the
// m-axis R2C of Theta, written straight into the x-update's spectrum layout.
// Theta never goes to HBM, which removes 8 of the iteration's bytes per voxel
// and one launch.
//
// A workgroup owns SR_ROWS whole rows along m (one wavefront per row) and
// marches along s through a chunk of planes, as the tiled stencil does:
//   - x of the rows n0-1 .. n0+SR_ROWS is staged in LDS (three rotating plane
//     buffers; m wraps inside the row, so no m ring is needed);
//   - nu_new, u', d' are formed for the tile and for row n0-1, whose
//     n-components feed L^T at row n0; a lane owns M/64 adjacent points of
//     its row, so the m-neighbour values L^T needs are its own points but
//     for the first, which comes from the lane to the left by a cross-lane
//     shuffle;
//   - Theta of the plane's rows goes into the plane buffer not in use, which
//     is then transformed along m as a half-length complex FFT and written out.
// The pointwise arithmetic is that of the tiled stencil (stencil_core.h) and
// the transform that of the row kernel (fft_core.h), so the spectrum matches
// the separate stencil + R2C path bit for bit.
#include "fft_core.h"
#include "reduce.h"

// No FMA contraction in the stencil arithmetic (see stencil_core.h); the FFT
// helpers above never contract either.
#pragma clang fp contract(off)
#include "stencil_core.h"

namespace sr3d {

constexpr int SR_ROWS = kThreads / 64;  // rows per tile = wavefronts per workgroup

template <int M>
struct SRGeom {
  static constexpr int CH = M / 64;                  // own points per lane and plane
  static constexpr int H = M / 2, MH = M / 2 + 1;    // half length, half spectrum
  static constexpr int XROWS = SR_ROWS + 2;          // x rows n0-1 .. n0+SR_ROWS
  static constexpr int XPLANE = XROWS * M;           // floats per x plane buffer
  static constexpr int XPT = (XPLANE + kThreads - 1) / kThreads;
  static constexpr int FPLANE = (SR_ROWS + 1) * M;   // n-components: row n0-1 and the tile
  static constexpr int FPT = (M + kThreads - 1) / kThreads;  // row n0-1 points per thread
  static constexpr int TP = SR_ROWS + 1;             // FFT buffer: line pitch
  static_assert(M % 64 == 0, "whole wavefront rows");
  static_assert(H * TP * 2 <= XPLANE, "the FFT buffer fits one x plane buffer");
};

// The n consecutive floats at p (16-byte aligned for n = 4, 8-byte for n = 2)
// as one LDS access.
template <int n>
__device__ __forceinline__ void lds_run(const float *p, float (&v)[n]) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  if constexpr (n == 4) {
    const f32x4 r = *reinterpret_cast<const f32x4 *>(p);
    v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
  } else if constexpr (n == 2) {
    const f32x2 r = *reinterpret_cast<const f32x2 *>(p);
    v[0] = r.x; v[1] = r.y;
  } else {
#pragma unroll
    for (int i = 0; i < n; ++i) v[i] = p[i];
  }
}

// Tile b of the plan; the residual sums go to partial slot `slot`.
template <int M, typename Acc, bool ANISO>
__device__ __forceinline__ void stencil_r2c_body(const AdmmStencilArgs &a, const StencilPlan &pl,
                                                 float2 *__restrict__ spec,
                                                 const int *__restrict__ kofp, int pitch,
                                                 const float2 *__restrict__ twh,
                                                 const float2 *__restrict__ twm, int b,
                                                 int slot) {
  using G = SRGeom<M>;
  constexpr int CH = G::CH, H = G::H, MH = G::MH, XPLANE = G::XPLANE, XPT = G::XPT;
  constexpr int FPT = G::FPT, TP = G::TP;
  __shared__ __align__(16) float xs[3][XPLANE];
  __shared__ float fw[G::FPLANE], fd[G::FPLANE], fu[G::FPLANE];  // n-components
  __shared__ float2 stw[H], stwm[MH];
  __shared__ int sperm[MH];
  __shared__ Acc sh[6 * 4];

  const int S = a.S, N = a.N;
  // Element offsets below 2^30 (the host checks the volume), so byte offsets
  // fit 32 bits; the three state components have base pointers of their own.
  const uint32_t NT = (uint32_t)S * N * M;
  const uint32_t plane = (uint32_t)N * M;
  const float *const nui0 = a.nu_in, *const nui1 = a.nu_in + NT, *const nui2 = a.nu_in + 2 * (size_t)NT;
  float *const nuo0 = a.nu_out, *const nuo1 = a.nu_out + NT, *const nuo2 = a.nu_out + 2 * (size_t)NT;
  const int tn = b % pl.tiles_n, ch = b / pl.tiles_n;
  const int n0 = tn * SR_ROWS;
  const int s0 = ch * pl.L;
  const int s1 = min(s0 + pl.L, S);
  const int tid = threadIdx.x, lane = tid & 63, row = tid >> 6;

  stage_twiddles<H>(stw, twh);
  for (int i = tid; i < MH; i += kThreads) {
    stwm[i] = twm[i];
    sperm[i] = kofp ? kofp[i] : i;
  }

  // x ring: ring row rr holds global row (n0 - 1 + rr) mod N. Element
  // r = tid + k kThreads of a plane is (r / M, r % M); when M is a multiple of
  // kThreads its row is the same across the workgroup, and only the row
  // starts are kept (scalars).
  constexpr bool kRowUniform = M % kThreads == 0;
  int xrow[G::XROWS];
#pragma unroll
  for (int rr = 0; rr < G::XROWS; ++rr) xrow[rr] = ((n0 - 1 + rr) % N + N) % N * M;
  int roff[kRowUniform ? 1 : XPT];
  if constexpr (!kRowUniform) {
#pragma unroll
    for (int k = 0; k < XPT; ++k) {
      const int r = tid + k * kThreads;
      const int rr = r / M, m = r % M;
      roff[k] = (r < XPLANE) ? ((n0 - 1 + rr) % N + N) % N * M + m : 0;
    }
  }
  auto ring_off = [&](int k) {
    if constexpr (kRowUniform)
      return xrow[(k * kThreads) / M] + (k * kThreads) % M + tid;
    else
      return roff[k];
  };
  // Own points: row `row` of the tile, m = CH lane + c (CH consecutive points
  // per lane, so their loads, stores and LDS accesses are adjacent).
  const int gn = (n0 + row) % N;
  const bool rval = n0 + row < N;
  // Row n0-1 points: m = tid + kThreads j (< M).
  const int fn = ((n0 - 1) % N + N) % N;

  auto ring_fetch = [&](int sp, float *xr) {
    const uint32_t base = (uint32_t)(((sp % S) + S) % S) * plane;
#pragma unroll
    for (int k = 0; k < XPT; ++k)
      xr[k] = (XPLANE % kThreads == 0 || tid + k * kThreads < XPLANE)
                  ? ld_off(a.x, base + (uint32_t)ring_off(k))
                  : 0.f;
  };
  auto ring_store = [&](int buf, const float *xr) {
#pragma unroll
    for (int k = 0; k < XPT; ++k)
      if (XPLANE % kThreads == 0 || tid + k * kThreads < XPLANE) xs[buf][tid + k * kThreads] = xr[k];
  };
  // nu_old at the own points (CH) and the row n0-1 points (FPT) of plane sp;
  // the own points' state is streamed (non-temporal loads, and stores of
  // nu_new), the row n0-1 points, which the tile above reads too, are not
  auto nu_fetch = [&](int sp, float (*o)[3]) {
    const uint32_t sb = (uint32_t)(((sp % S) + S) % S) * plane;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const uint32_t v = sb + (uint32_t)(gn * M + CH * lane + c);
      o[c][0] = ld_off_nt(nui0, v);
      o[c][1] = ld_off_nt(nui1, v);
      o[c][2] = ld_off_nt(nui2, v);
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int m = tid + kThreads * j;
      const uint32_t v = sb + (uint32_t)(fn * M + (m < M ? m : 0));
      o[CH + j][0] = ld_off(nui0, v);
      o[CH + j][1] = ld_off(nui1, v);
      o[CH + j][2] = ld_off(nui2, v);
    }
  };
  // LDS index of the point (ring row rr, m) and of its m and n successors
  auto idx = [](int rr, int m) { return rr * M + m; };
  auto idx_m1 = [](int rr, int m) { return rr * M + (m + 1 == M ? 0 : m + 1); };

  // x at the lane's own points of a plane (xa), at their n successors (xb)
  // and s successors (xz), from the plane buffers xc (this plane) and xn (the
  // next); the m successor of the last point is the next lane's first point.
  auto own_x = [&](const float *xc, const float *xn, float (&xa)[CH], float (&xb)[CH],
                   float (&xz)[CH], float &xl) {
    lds_run<CH>(xc + (row + 1) * M + CH * lane, xa);
    lds_run<CH>(xc + (row + 2) * M + CH * lane, xb);
    lds_run<CH>(xn + (row + 1) * M + CH * lane, xz);
    xl = lane_next(xa[0]);
  };

  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float pw[CH], pd[CH], pu[CH];  // s-components at the previous plane
  float xr[XPT];
  float nuc[CH + FPT][3], nun[CH + FPT][3];

  // Prologue: plane s0 - 1 (its s-components feed L^T at plane s0).
  {
    float xp[XPT], nup[CH + FPT][3];
    ring_fetch(s0 - 1, xp);
    ring_fetch(s0, xr);
    nu_fetch(s0 - 1, nup);
    ring_store(0, xp);
    ring_store(1, xr);
    ring_fetch(s0 + 1, xr);
    nu_fetch(s0, nuc);
    __syncthreads();
    float xa[CH], xb[CH], xz[CH], xl;
    own_x(xs[0], xs[1], xa, xb, xz, xl);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      PointQ q;
      point_update_x<ANISO>(xa[c], c + 1 < CH ? xa[c + 1] : xl, xb[c], xz[c], nup[c][0], nup[c][1],
                            nup[c][2], a.thr, q);
      pw[c] = q.w[2];
      pd[c] = q.d[2];
      pu[c] = q.du[2];
    }
  }

  float2 *out = spec;
  for (int sp = s0; sp < s1; ++sp) {
    const int bc = (sp - s0 + 1) % 3, bn = (sp - s0 + 2) % 3, bz = (sp - s0) % 3;
    __syncthreads();     // the previous plane's FFT buffer (buffer bn now) is read out
    ring_store(bn, xr);  // plane sp + 1
    if (sp + 1 < s1) {
      ring_fetch(sp + 2, xr);
      nu_fetch(sp + 1, nun);
    }
    __syncthreads();
    const uint32_t sb = (uint32_t)sp * plane;
    float mw[CH], md[CH], mu[CH];     // m-components at the own points
    float tw[CH], td[CH], tu[CH];     // s-term minus the point's own sum
    float fnw[CH], fnd[CH], fnu[CH];  // n-components
    float nn0[CH], nn1[CH], nn2[CH];  // nu_new
    float xa[CH], xb[CH], xz[CH], xl;
    own_x(xs[bc], xs[bn], xa, xb, xz, xl);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      PointQ q;
      point_update_x<ANISO>(xa[c], c + 1 < CH ? xa[c + 1] : xl, xb[c], xz[c], nuc[c][0], nuc[c][1],
                            nuc[c][2], a.thr, q);
      fnw[c] = q.w[1];
      fnd[c] = q.d[1];
      fnu[c] = q.du[1];
      nn0[c] = q.nn[0];
      nn1[c] = q.nn[1];
      nn2[c] = q.nn[2];
      mw[c] = q.w[0];
      md[c] = q.d[0];
      mu[c] = q.du[0];
      tw[c] = pw[c] - (q.w[0] + q.w[1] + q.w[2]);
      td[c] = pd[c] - (q.d[0] + q.d[1] + q.d[2]);
      tu[c] = pu[c] - (q.du[0] + q.du[1] + q.du[2]);
      pw[c] = q.w[2];
      pd[c] = q.d[2];
      pu[c] = q.du[2];
      if (rval) point_stats<ANISO>(q, acc);
    }
    // The lane's CH points are adjacent: each array is written as one run.
    {
      const int f0 = (row + 1) * M + CH * lane;
#pragma unroll
      for (int c = 0; c < CH; ++c) fw[f0 + c] = fnw[c];
#pragma unroll
      for (int c = 0; c < CH; ++c) fd[f0 + c] = fnd[c];
#pragma unroll
      for (int c = 0; c < CH; ++c) fu[f0 + c] = fnu[c];
    }
    if (rval) {
      const uint32_t v = sb + (uint32_t)(gn * M + CH * lane);
#pragma unroll
      for (int c = 0; c < CH; ++c) st_off_nt(nuo0, v + c, nn0[c]);
#pragma unroll
      for (int c = 0; c < CH; ++c) st_off_nt(nuo1, v + c, nn1[c]);
#pragma unroll
      for (int c = 0; c < CH; ++c) st_off_nt(nuo2, v + c, nn2[c]);
    }
#pragma unroll
    for (int j = 0; j < FPT; ++j) {
      const int m = tid + kThreads * j;
      if (M % kThreads == 0 || m < M) {
        PointQ q;
        point_update_at<ANISO>(xs[bc], xs[bn], idx(0, m), idx_m1(0, m), idx(1, m),
                               nuc[CH + j][0], nuc[CH + j][1], nuc[CH + j][2], a.thr, q);
        fw[m] = q.w[1];
        fd[m] = q.d[1];
        fu[m] = q.du[1];
      }
    }
    // The m-neighbour (m - 1, wrapping) of point c > 0 of a lane is its point
    // c - 1; that of point 0 is the last point of lane l - 1, and for lane 0
    // that of lane 63 (m = M - 1): a rotation of the wavefront by one lane.
    float lw[CH], ld[CH], lu[CH];
    lw[0] = lane_prev(mw[CH - 1]);
    ld[0] = lane_prev(md[CH - 1]);
    lu[0] = lane_prev(mu[CH - 1]);
#pragma unroll
    for (int c = 1; c < CH; ++c) {
      lw[c] = mw[c - 1];
      ld[c] = md[c - 1];
      lu[c] = mu[c - 1];
    }
    __syncthreads();
    float *z = xs[bz];  // FFT buffer: z[2 (i TP + t) + e] = Theta[t][2 i + e]
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int m = CH * lane + c;
      const int fi = row * M + m;  // the point's n-neighbour (row above)
      // (L^T z)[i] = (z_m[i - e_m] + z_n[i - e_n]) + (z_s[i - e_s] - sum_a z_a[i])
      const float ltw = (lw[c] + fw[fi]) + tw[c];
      const float ltd = (ld[c] + fd[fi]) + td[c];
      const float ltu = (lu[c] + fu[fi]) + tu[c];
      z[2 * ((m >> 1) * TP + row) + (m & 1)] = ltw;
      if (rval) {
        acc[4] = fmaf(ltu, ltu, acc[4]);
        acc[5] = fmaf(ltd, ltd, acc[5]);
      }
    }
#pragma unroll
    for (int k = 0; k < CH + FPT; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) nuc[k][c] = nun[k][c];
    __syncthreads();
    float2 *z2 = reinterpret_cast<float2 *>(z);
    fft_passes<H, SR_ROWS, TP, 0, 1>(z2, stw);
    for (int w = tid; w < MH * SR_ROWS; w += kThreads) {
      const int p = w % MH, t = w / MH;
      if (n0 + t < N) {
        const int k = sperm[p];
        st_off2(out, ((uint32_t)sp * N + n0 + t) * (uint32_t)pitch + p,
                r2c_post(z2[(k % H) * TP + t], z2[((H - k) % H) * TP + t], stwm[k]));
      }
    }
  }
  Acc acc_t[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) acc_t[q] = (Acc)acc[q];
  block_reduce_n<Acc>(acc_t, 6, sh);
  if (tid == 0) {
    Acc *p = reinterpret_cast<Acc *>(a.part);
    for (int q = 0; q < 6; ++q) p[(long)q * pl.blocks + slot] = acc_t[q];
  }
}

template <int M, typename Acc, bool ANISO>
__global__ __launch_bounds__(kThreads) void k_admm_stencil_r2c(AdmmStencilArgs a, StencilPlan pl,
                                                               float2 *__restrict__ spec,
                                                               const int *__restrict__ kofp,
                                                               int pitch,
                                                               const float2 *__restrict__ twh,
                                                               const float2 *__restrict__ twm) {
  if (a.done && *a.done) return;
  stencil_r2c_body<M, Acc, ANISO>(a, pl, spec, kofp, pitch, twh, twm,
                                  xcd_tile(blockIdx.x, pl.blocks), blockIdx.x);
}

// Batch: item (volume, tile) of the volumes with row length M; iteration k
// reads nu[(k-1)&1] and writes nu[k&1].
template <int M, typename Acc, bool ANISO>
__global__ __launch_bounds__(kThreads) void k_admm_stencil_r2c_batch(
    const BatchStencilDesc *__restrict__ descs, const int2 *__restrict__ items, int k,
    const float2 *__restrict__ twh, const float2 *__restrict__ twm) {
  const int2 it = items[blockIdx.x];
  const BatchStencilDesc d = descs[it.x];
  if (d.a.done && *d.a.done) return;
  AdmmStencilArgs a = d.a;
  // A select, not an index into the local copy (which would put it in scratch).
  float *const nu0 = d.nu[0], *const nu1 = d.nu[1];
  a.nu_in = (k & 1) ? nu0 : nu1;
  a.nu_out = (k & 1) ? nu1 : nu0;
  stencil_r2c_body<M, Acc, ANISO>(a, d.pl, d.spec, d.kofp, d.pitch, twh, twm, it.y, it.y);
}

// Row lengths where the fused kernel is faster than the tiled stencil and
// the separate R2C together. Longer rows hold 6 or 8 points per lane and
// plane, 222 VGPRs at m = 384 and 256 plus 19 AGPRs at m = 512 (two and one
// wavefronts per SIMD), and measured slower: 304 against 200 us at m = 384,
// 890 against 588 us at m = 512.
#define SR3D_STENCIL_R2C_M(X) X(64) X(128) X(192) X(256)

bool stencil_r2c_supported(int M) {
  switch (M) {
#define SR3D_CASE(L) case L:
    SR3D_STENCIL_R2C_M(SR3D_CASE)
#undef SR3D_CASE
    return true;
    default:
      return false;
  }
}

bool stencil_r2c_fits(int S, int N, int M, int pitch) {
  const uint64_t nt = (uint64_t)S * N * M, rows = (uint64_t)S * N;
  return stencil_r2c_supported(M) && nt * 4 < (1ull << 32) && rows * pitch * 8 < (1ull << 32);
}

StencilPlan stencil_r2c_plan(int S, int N, int M) {
  StencilPlan p;
  p.tiles_m = 1;
  p.tiles_n = (N + SR_ROWS - 1) / SR_ROWS;
  // One round of workgroups over the 256 CUs at the occupancy the row
  // length allows (registers and LDS grow with M), 2..32 planes each.
  const long target = M <= 128 ? 1024 : 768;
  long L = ((long)S * p.tiles_n + target - 1) / target;
  if (L < 2) L = 2;
  if (L > 32) L = 32;
  if (L > S) L = S;
  p.L = (int)L;
  p.chunks = (S + p.L - 1) / p.L;
  p.blocks = p.tiles_n * p.chunks;
  return p;
}

template <int M, bool ANISO>
static void launch_sr_t(const AdmmStencilArgs &a, const StencilPlan &pl, float2 *spec,
                        const int *kofp, int pitch, bool fp64, hipStream_t st) {
  const float2 *twh = twiddles(M / 2), *twm = twiddles(M);
  if (fp64)
    hipLaunchKernelGGL((k_admm_stencil_r2c<M, double, ANISO>), dim3(pl.blocks), dim3(kThreads), 0,
                       st, a, pl, spec, kofp, pitch, twh, twm);
  else
    hipLaunchKernelGGL((k_admm_stencil_r2c<M, float, ANISO>), dim3(pl.blocks), dim3(kThreads), 0,
                       st, a, pl, spec, kofp, pitch, twh, twm);
}

template <int M>
static void launch_sr(const AdmmStencilArgs &a, const StencilPlan &pl, float2 *spec,
                      const int *kofp, int pitch, bool fp64, hipStream_t st) {
  if (a.aniso) launch_sr_t<M, true>(a, pl, spec, kofp, pitch, fp64, st);
  else launch_sr_t<M, false>(a, pl, spec, kofp, pitch, fp64, st);
}

template <int M, bool ANISO>
static void launch_srb_t(const BatchStencilDesc *descs, const int2 *items, int nitems, int k,
                         bool fp64, hipStream_t st) {
  const float2 *twh = twiddles(M / 2), *twm = twiddles(M);
  if (fp64)
    hipLaunchKernelGGL((k_admm_stencil_r2c_batch<M, double, ANISO>), dim3(nitems), dim3(kThreads),
                       0, st, descs, items, k, twh, twm);
  else
    hipLaunchKernelGGL((k_admm_stencil_r2c_batch<M, float, ANISO>), dim3(nitems), dim3(kThreads),
                       0, st, descs, items, k, twh, twm);
}

hipError_t admm_stencil_r2c_batch(int M, const BatchStencilDesc *descs, const int2 *items,
                                  int nitems, int k, bool fp64, bool aniso, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  if (!stencil_r2c_supported(M) || !twiddles(M) || !twiddles(M / 2)) return hipErrorInvalidValue;
  switch (M) {
#define SR3D_CASE(L)                                                        \
  case L:                                                                   \
    if (aniso) launch_srb_t<L, true>(descs, items, nitems, k, fp64, st);   \
    else launch_srb_t<L, false>(descs, items, nitems, k, fp64, st);        \
    break;
    SR3D_STENCIL_R2C_M(SR3D_CASE)
#undef SR3D_CASE
  }
  return hipGetLastError();
}

hipError_t admm_stencil_r2c(const AdmmStencilArgs &a, float2 *spec, const int *kofp, int pitch,
                            bool fp64, hipStream_t st) {
  if (!stencil_r2c_supported(a.M) || !a.x || !a.nu_in || !a.nu_out || !a.part || !spec ||
      pitch < a.M / 2 + 1 || !twiddles(a.M) || !twiddles(a.M / 2))
    return hipErrorInvalidValue;
  const StencilPlan pl = stencil_r2c_plan(a.S, a.N, a.M);
  prof_begin(kStStencilR2c, st);
  switch (a.M) {
#define SR3D_CASE(L)                                       \
  case L:                                                  \
    launch_sr<L>(a, pl, spec, kofp, pitch, fp64, st);      \
    break;
    SR3D_STENCIL_R2C_M(SR3D_CASE)
#undef SR3D_CASE
  }
  const hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

}  // namespace sr3d
