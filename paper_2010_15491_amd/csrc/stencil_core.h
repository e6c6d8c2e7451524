// Pointwise pieces of the ADMM stencil (Algorithm 1 steps 5b, 5c) shared by
// the stencil kernels.
//
// Included after the file's `#pragma clang fp contract(off)`: the compiler
// fuses no product into a sum, and the fused multiply-adds used here are
// explicit (fmaf), so all kernels built from these pieces (and the resume
// path) produce the same bits for the same point.
#pragma once

#include "sr3d_internal.h"

namespace sr3d {

template <typename T>
__device__ __forceinline__ void block_reduce_n(T *v, int n, T *sh /* [n][4] */) {
  for (int q = 0; q < n; ++q) {
    T s = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    v[q] = s;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
    for (int q = 0; q < n; ++q) sh[q * 4 + wid] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < n; ++q) v[q] = sh[q * 4 + 0] + sh[q * 4 + 1] + sh[q * 4 + 2] + sh[q * 4 + 3];
}

// Global loads and stores at a 32-bit byte offset from a base pointer held in
// scalar registers (the hardware's scalar-base addressing: no 64-bit address
// arithmetic per lane). Callers keep every offset below 4 GiB.
__device__ __forceinline__ float ld_off(const float *base, uint32_t i) {
  return *(__attribute__((address_space(1))) const float *)(
      (__attribute__((address_space(1))) const char *)base + (i << 2));
}
__device__ __forceinline__ void st_off(float *base, uint32_t i, float v) {
  *(__attribute__((address_space(1))) float *)((__attribute__((address_space(1))) char *)base +
                                               (i << 2)) = v;
}
// The same as non-temporal accesses, for streams that are not read again
// before much more data has passed through the caches (the ADMM state, read
// and written once per iteration): they leave the last-level cache to the
// spectrum and the Lambda table, which the next kernels read.
__device__ __forceinline__ float ld_off_nt(const float *base, uint32_t i) {
  return __builtin_nontemporal_load((__attribute__((address_space(1))) const float *)(
      (__attribute__((address_space(1))) const char *)base + (i << 2)));
}
__device__ __forceinline__ void st_off_nt(float *base, uint32_t i, float v) {
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) float *)(
                                     (__attribute__((address_space(1))) char *)base + (i << 2)));
}
__device__ __forceinline__ void st_off2(float2 *base, uint32_t i, float2 v) {
  const uint64_t bits = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
  *(__attribute__((address_space(1))) uint64_t *)((__attribute__((address_space(1))) char *)base +
                                                  (i << 3)) = bits;
}

// The value of lane (l - 1) mod 64 of the wavefront: a DPP rotation of the
// whole wavefront right by one lane (no LDS traffic).
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C /* wave_ror:1 */,
                                                    0xF, 0xF, false));
}

// The value of lane (l + 1) mod 64: a DPP rotation of the wavefront left by
// one lane.
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134 /* wave_rol:1 */,
                                                    0xF, 0xF, false));
}

// Workgroup b of nb is dispatched to XCD b % 8; give every XCD a contiguous
// range of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, l = b >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Isotropic shrink (Algorithm 1 step 5b): u = a max(|a| - thr, 0) / |a|,
// written as a max(1 - thr / |a|, 0) with the hardware reciprocal square
// root; a = 0 gives u = 0.
__device__ __forceinline__ void shrink3(float a0, float a1, float a2, float thr, float &u0,
                                        float &u1, float &u2) {
  const float n2 = fmaf(a2, a2, fmaf(a1, a1, a0 * a0));
  const float s = n2 > 0.f ? fmaxf(fmaf(-thr, __builtin_amdgcn_rsqf(n2), 1.f), 0.f) : 0.f;
  u0 = a0 * s;
  u1 = a1 * s;
  u2 = a2 * s;
}

// Anisotropic TV (sum over voxels and components of |(L x)_{j,a}|, one of the
// other regularisers the same x-step serves, Sec. III-B): step 5b becomes the
// soft threshold of every component, u = sign(a) max(|a| - thr, 0).
__device__ __forceinline__ float shrink1(float a, float thr) {
  return copysignf(fmaxf(fabsf(a) - thr, 0.f), a);
}

template <bool ANISO>
__device__ __forceinline__ void shrink_tv(float a0, float a1, float a2, float thr, float &u0,
                                          float &u1, float &u2) {
  if constexpr (ANISO) {
    u0 = shrink1(a0, thr);
    u1 = shrink1(a1, thr);
    u2 = shrink1(a2, thr);
  } else {
    shrink3(a0, a1, a2, thr, u0, u1, u2);
  }
}

// Quantities of one point after the update: w = u' - d', d', du = u' - u.
struct PointQ {
  float w[3], d[3], du[3];
  float l[3], u[3];   // L x and u' (for the primal residual sums)
  float nn[3];        // nu_new
};

// One point of the update from x at the point (xi), at its m, n and s
// successors (xm, xn, xs), and nu_old.
template <bool ANISO>
__device__ __forceinline__ void point_update_x(float xi, float xm, float xn, float xs, float o0,
                                               float o1, float o2, float thr, PointQ &q) {
  q.l[0] = xm - xi;
  q.l[1] = xn - xi;
  q.l[2] = xs - xi;
  float uo0, uo1, uo2;
  shrink_tv<ANISO>(o0, o1, o2, thr, uo0, uo1, uo2);
  q.nn[0] = q.l[0] + (o0 - uo0);
  q.nn[1] = q.l[1] + (o1 - uo1);
  q.nn[2] = q.l[2] + (o2 - uo2);
  shrink_tv<ANISO>(q.nn[0], q.nn[1], q.nn[2], thr, q.u[0], q.u[1], q.u[2]);
  const float uo[3] = {uo0, uo1, uo2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    q.d[c] = q.nn[c] - q.u[c];
    q.w[c] = q.u[c] - q.d[c];
    q.du[c] = q.u[c] - uo[c];
  }
}

// The same with x read from plane buffers: the point at xc[ri], its m and n
// successors at xc[rm], xc[rn], its s successor at xn[ri].
template <bool ANISO>
__device__ __forceinline__ void point_update_at(const float *xc, const float *xn, int ri, int rm,
                                                int rn, float o0, float o1, float o2, float thr,
                                                PointQ &q) {
  point_update_x<ANISO>(xc[ri], xc[rm], xc[rn], xn[ri], o0, o1, o2, thr, q);
}

// The point's terms of the residual sums: |Lx - u'|^2, |Lx|^2, |u'|^2 and
// the regulariser's |(Lx)_j| (accumulated with fused multiply-adds; these
// sums feed only the stopping test and the objective).
template <bool ANISO>
__device__ __forceinline__ void point_stats(const PointQ &q, float *acc) {
  const float r0 = q.l[0] - q.u[0], r1 = q.l[1] - q.u[1], r2 = q.l[2] - q.u[2];
  acc[0] = fmaf(r2, r2, fmaf(r1, r1, fmaf(r0, r0, acc[0])));
  const float l2 = fmaf(q.l[2], q.l[2], fmaf(q.l[1], q.l[1], q.l[0] * q.l[0]));
  acc[1] += l2;
  acc[2] = fmaf(q.u[2], q.u[2], fmaf(q.u[1], q.u[1], fmaf(q.u[0], q.u[0], acc[2])));
  if constexpr (ANISO)
    acc[3] += fabsf(q.l[0]) + fabsf(q.l[1]) + fabsf(q.l[2]);
  else
    acc[3] += l2 > 0.f ? l2 * __builtin_amdgcn_rsqf(l2) : 0.f;
}

}  // namespace sr3d
