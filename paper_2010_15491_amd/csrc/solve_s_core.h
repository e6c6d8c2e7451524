// Device code of the fused x-update along s (see solve_s.hip for the method):
// unit helpers, the kernel template and its launchers. Included by the
// translation units that instantiate the kernel for groups of s-lengths, so
// the instances compile in parallel.
#pragma once

#include "fft_core.h"

namespace sr3d {

// Lines per workgroup: as many as fit two workgroups in a CU's 160 KB of LDS
// (lines, twiddles, |sigma_s|^2 table and side tables), at most 64, rounded
// down to a multiple of 8 so that units of whole (2-column class x 4-row)
// blocks fill the tile (32 of 32 lines at s = 256, d = 2^3, instead of 32 or
// 36 of 37).
constexpr int solve_tile(int S) {
  const int t = (81920 - 12 * S - 2048) / (8 * S);
  return t > 64 ? 64 : t / 8 * 8;
}

// ---------------------------------------------------------------------------
// Device
// ---------------------------------------------------------------------------

// Global-memory views of pointers read from a descriptor in memory (the
// compiler cannot infer their address space and would emit flat accesses,
// which share the LDS wait counter).
typedef __attribute__((address_space(1))) const float cgfloat;
typedef __attribute__((address_space(1))) const int cgint;
typedef __attribute__((address_space(1))) const uint64_t cgu64;
typedef __attribute__((address_space(1))) uint64_t gu64;

__device__ __forceinline__ float2 u64_f2(uint64_t v) {
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}
__device__ __forceinline__ uint64_t f2_u64(float2 v) {
  return (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
}
// complex value at byte offset `off` from global base `b`
__device__ __forceinline__ float2 gld2(const void *b, uint32_t off) {
  return u64_f2(*(cgu64 *)((__attribute__((address_space(1))) const char *)b + off));
}
__device__ __forceinline__ void gst2(void *b, uint32_t off, float2 v) {
  *(gu64 *)((__attribute__((address_space(1))) char *)b + off) = f2_u64(v);
}
// two complex values (16 bytes) at byte offset `off`
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 gld4(const void *b, uint32_t off) {
  return *(__attribute__((address_space(1))) const f32x4 *)((__attribute__((address_space(1))) const char *)b + off);
}
__device__ __forceinline__ void gst4(void *b, uint32_t off, f32x4 v) {
  *(__attribute__((address_space(1))) f32x4 *)((__attribute__((address_space(1))) char *)b + off) = v;
}

__device__ __forceinline__ float2 s_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 s_conj(float2 a) { return make_float2(a.x, -a.y); }

template <typename T>
__device__ __forceinline__ T unit_sum(T v, T *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

__device__ __forceinline__ int solve_xcd_unit(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, l = b >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Group of slot `slot` of a unit whose m-block has nc classes (slots
// 0 .. 2 S_l nc - 1): returns false for an empty or skipped slot.
struct SlotGroup {
  int js, jn, jm, ji, ci;
  bool selfc;
};
__device__ __forceinline__ int block_classes(const int *mj, int CB) {
  int nc = 0;
  while (nc < CB && mj[nc] >= 0) ++nc;
  return nc;
}
// Slot = r1 * nc + ci with r1 = 2 js + ji.
__device__ __forceinline__ bool slot_group_at(const SolveSArgs &a, const int *mj, int ci, int r1,
                                              int j0, int j1, SlotGroup &g) {
  const int ji = r1 & 1, js = r1 >> 1;
  const int jm = mj[ci];
  if (jm < 0 || (ji && j1 < 0)) return false;
  const int jn = ji ? j1 : j0;
  bool selfc = false;
  if (jm == 0 || 2 * jm == a.Ml) {  // self-conjugate m class: keep one of j, -j
    const int jsn = js == 0 ? 0 : a.Sl - js, jnn = jn == 0 ? 0 : a.Nl - jn;
    const long lin = (long)js * a.Nl + jn, lnn = (long)jsn * a.Nl + jnn;
    if (lin > lnn) return false;
    selfc = lin == lnn;
  }
  g = SlotGroup{js, jn, jm, ji, ci, selfc};
  return true;
}
__device__ __forceinline__ bool slot_group(const SolveSArgs &a, const int *mj, int nc, int j0,
                                           int j1, int slot, SlotGroup &g) {
  return slot_group_at(a, mj, slot % nc, slot / nc, j0, j1, g);
}

// LDS side tables of a unit (sizes bound the plan: lines <= 64, classes per
// block * dr <= 64, rows <= 2 dc <= 64).
struct UnitTabs {
  int loff[64];     // global offset of line l within an s-plane, or -1
  int mj[64];       // class representatives j_m of the m-block (-1: none)
  int nc;           // classes in the m-block
  int mpos[64];     // (ci, a): line position of the stored rep of k_m, bit 30 = mirrored
  float gmv[64];    // (ci, a): |sigma_m(k_m)|^2
  int rowd[64];     // (ji, b): row of k_n
  int rowm[64];     // (ji, b): row of -k_n
  float gnv[64];    // (ji, b): |sigma_n(k_n)|^2
};

template <int S, int DM, bool EXACT, int GR, typename Acc>
__device__ __forceinline__ void solve_s_body(const SolveSArgs &a, int u,
                                             const float2 *__restrict__ tw, float2 *lds,
                                             float2 *stw, float *sgs, UnitTabs &ut, Acc *red) {
  constexpr int T = solve_tile(S), TP = T;
  const int gn = u / a.NB, bm = u - gn * a.NB;
  cgint *tab = (cgint *)a.tab;
  cgfloat *gmt = (cgfloat *)a.gm, *gnt = (cgfloat *)a.gn, *gst = (cgfloat *)a.gs;
  const int p0 = tab[a.o_p0 + bm], cnt = tab[a.o_cnt + bm];
  const int j0 = tab[a.o_nj + 2 * gn], j1 = tab[a.o_nj + 2 * gn + 1];
  const int nji = j1 < 0 ? 1 : 2;
  const int nlines = nji * a.dc * cnt;
  const long plane = (long)a.N * a.P;
  stage_twiddles<S>(stw, tw);
  for (int i = threadIdx.x; i < S; i += kThreads) sgs[i] = gst[i];
  {
    const int t = threadIdx.x;
    if (t < T) {
      int off = -1;
      if (t < nlines) {
        const int row = t / cnt, pp = t - row * cnt;
        const int ji = row / a.dc, b = row - ji * a.dc;
        off = ((ji ? j1 : j0) + b * a.Nl) * a.P + p0 + pp;
      }
      ut.loff[t] = off;
    }
    if (t < a.CB) ut.mj[t] = tab[a.o_mj + bm * a.CB + t];
    if (t == 0) {
      int nc = 0;
      while (nc < a.CB && tab[a.o_mj + bm * a.CB + nc] >= 0) ++nc;
      ut.nc = nc;
    }
    if (t < a.CB * a.dr) {
      const int ci = t / a.dr, ia = t - ci * a.dr;
      const int jm = tab[a.o_mj + bm * a.CB + ci];
      if (jm >= 0) {
        const int km = jm + ia * a.Ml;
        const bool direct = km < a.Mh;
        const int rm = direct ? km : a.M - km;
        ut.mpos[t] = (tab[a.Mh + rm] - p0) | (direct ? 0 : (1 << 30));
        ut.gmv[t] = gmt[km];
      }
    }
    if (t < nji * a.dc) {
      const int ji = t / a.dc, b = t - ji * a.dc;
      const int jn = ji ? j1 : j0;
      const int jnn = jn == 0 ? 0 : a.Nl - jn;
      const int jim = (jnn == j0) ? 0 : 1;
      const int bmir = (jn == 0) ? ((a.dc - b) % a.dc) : (a.dc - 1 - b);
      ut.rowd[t] = t;
      ut.rowm[t] = jim * a.dc + bmir;
      ut.gnv[t] = gnt[jn + b * a.Nl];
    }
  }
  __syncthreads();
  // Element w of the tile is (s, line) = (w / T, w % T), at lds[w]. All of a
  // thread's loads are issued before the first LDS store; lines past the
  // unit's load element 0 and are zeroed.
  constexpr int NE = (S * T + kThreads - 1) / kThreads;
  constexpr int NH = (NE + 1) / 2;  // loads in flight per thread: half the tile
  const uint32_t pl = (uint32_t)plane;
  // Where every row run of the unit has an even length and starts at an even
  // column, lines 2i and 2i + 1 are adjacent columns of one row: each thread
  // then moves pairs of them (16 bytes) with half the instructions.
  const bool pairs = ((cnt | p0 | a.P) & 1) == 0;
  constexpr int NP = (S * T / 2 + kThreads - 1) / kThreads;
  constexpr int NPH = (NP + 1) / 2;
  if (pairs) {
#pragma unroll
    for (int h = 0; h < NP; h += NPH) {
      f32x4 v[NPH];
#pragma unroll
      for (int k = 0; k < NPH; ++k) {
        const int w2 = threadIdx.x + (h + k) * kThreads;
        const int s = w2 / (T / 2), line = 2 * (w2 - s * (T / 2));
        const int off = (h + k < NP && w2 < S * T / 2) ? ut.loff[line] : -1;
        const f32x4 x =
            gld4(a.W, ((uint32_t)(off >= 0 ? s : 0) * pl + (uint32_t)(off >= 0 ? off : 0)) * 8u);
        v[k] = off >= 0 ? x : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int k = 0; k < NPH; ++k) {
        const int w2 = threadIdx.x + (h + k) * kThreads;
        if (h + k < NP && w2 < S * T / 2) reinterpret_cast<f32x4 *>(lds)[w2] = v[k];
      }
    }
  } else
#pragma unroll
  for (int h = 0; h < NE; h += NH) {
    float2 v[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int w = threadIdx.x + (h + k) * kThreads;
      const int s = w / T, line = w - s * T;
      const int off = (h + k < NE && w < S * T) ? ut.loff[line] : -1;
      const float2 x = gld2(a.W, ((uint32_t)(off >= 0 ? s : 0) * pl + (uint32_t)(off >= 0 ? off : 0)) * 8u);
      v[k] = off >= 0 ? x : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int w = threadIdx.x + (h + k) * kThreads;
      if (h + k < NE && w < S * T) lds[w] = v[k];
    }
  }
  __syncthreads();
  fft_passes<S, T, TP, 0, 1>(lds, stw);

  // Solve. A group of up to DM members is spread over LANES = DM / 8
  // consecutive lanes, 8 members each (lane sub holds members 8 sub .. 8 sub
  // + 7), so every instance keeps the register footprint of the 8-member
  // one. Every LDS entry is read and written by one lane only: a member's own
  // entry and its mirror belong to it alone.
  // Group size: a compile-time constant in the EXACT instances (D = DM), so
  // the member loops unroll into straight-line code.
  constexpr int LANES = DM / 8, DL = DM / LANES;
  const int D = EXACT ? DM : a.D;
  const float fd = (float)D;
  const int sub = (int)threadIdx.x & (LANES - 1), gi = (int)threadIdx.x / LANES;
  const int gbase = ((int)threadIdx.x & 63) - sub;  // lane of member 0's owner
  constexpr int GT = kThreads / LANES;              // groups in flight per workgroup
  // member 8 sub -> (a, b, c) counters along m, n, s
  // Rates along m and n: compile-time constants (both GR) in the instances
  // specialised for the common rates, where every member's table indices
  // then fold away.
  const int GDR = GR ? GR : a.dr, GDC = GR ? GR : a.dc;
  const int m0 = sub * DL, ia0 = m0 % GDR, ib0 = (m0 / GDR) % GDC, ic0 = m0 / (GDR * GDC);
  Acc resid = 0;
  // Lambda of member q of slot i at Lu + (q gmax + i) 8 bytes, Y of slot i at
  // Yu + 8 i: 32-bit byte offsets from the unit's bases (at most
  // 32 members x 2^16 slots x 8 bytes).
  const char *Lu = (const char *)a.Lg + (size_t)u * D * a.gmax * 8;
  const char *Yu = (const char *)a.Yg + (size_t)u * a.gmax * 8;
  const uint32_t gstr = (uint32_t)a.gmax * 8u, lo0 = (uint32_t)m0 * gstr;
  // Lambda and Y of the next slot are loaded while the current one is solved.
  float2 lnext[DL], ynext = make_float2(0.f, 0.f);
  const int nc = ut.nc, gcount = a.Sl * 2 * nc;  // slots of this unit
  if (gi < gcount) {
    ynext = gld2(Yu, (uint32_t)gi * 8u);
#pragma unroll
    for (int q = 0; q < DL; ++q)
      if (EXACT || m0 + q < D) lnext[q] = gld2(Lu, lo0 + q * gstr + (uint32_t)gi * 8u);
  }
  // slot -> (ci, r1) advanced incrementally: GT = dq * nc + dr
  const int dq = GT / nc, dr = GT - dq * nc;
  int sci = gi % nc, sr1 = gi / nc;
  for (int slot = gi; slot < gcount; slot += GT) {
    const int ci = sci;
    float2 lcur[DL];
#pragma unroll
    for (int q = 0; q < DL; ++q) lcur[q] = lnext[q];
    const float2 Yj = ynext;
    const int nslot = slot + GT;
    if (nslot < gcount) {
      ynext = gld2(Yu, (uint32_t)nslot * 8u);
#pragma unroll
      for (int q = 0; q < DL; ++q)
        if (EXACT || m0 + q < D) lnext[q] = gld2(Lu, lo0 + q * gstr + (uint32_t)nslot * 8u);
    }
    SlotGroup g;
    const bool ok = slot_group_at(a, ut.mj, ci, sr1, j0, j1, g);
    sci += dr;
    sr1 += dq;
    if (sci >= nc) {
      sci -= nc;
      ++sr1;
    }
    if (!ok) continue;  // the same for every lane of the group
    // Members: Lambda, B = conj(Lambda) Y + mu W, A = mu G, the LDS index of
    // the stored entry (li >= 0: the member itself, else -1-index of its
    // mirror) and, for a stored member whose -k is stored as well and belongs
    // to the partner group, the LDS index of -k (mi, else -1).
    float2 B[DL];
    float A[DL];
    int li[DL], mi[DL];
    int ia = ia0, ib = ib0, ic = ic0;
#pragma unroll
    for (int q = 0; q < DL; ++q) {
      if (EXACT || m0 + q < D) {
        const int ks = g.js + ic * a.Sl;
        const int mp = ut.mpos[g.ci * GDR + ia];
        const bool direct = (mp & (1 << 30)) == 0;
        const int nrow = g.ji * GDC + ib;
        const int rs = ks == 0 ? 0 : S - ks;
        const int mirror = rs * TP + ut.rowm[nrow] * cnt + (mp & ~(1 << 30));
        const int idx = direct ? ks * TP + nrow * cnt + mp : mirror;
        float2 w = lds[idx];
        if (!direct) w.y = -w.y;
        const float2 l = lcur[q];
        const float Aq = a.mu * (sgs[ks] + ut.gnv[nrow] + ut.gmv[g.ci * GDR + ia]);
        const float2 cb = s_mul(s_conj(l), Yj);
        B[q] = make_float2(cb.x + a.mu * w.x, cb.y + a.mu * w.y);
        A[q] = Aq;
        li[q] = direct ? idx : -1 - idx;
        const int km = g.jm + ia * a.Ml;
        mi[q] = (direct && !g.selfc && (km == 0 || 2 * km == a.M)) ? mirror : -1;
        if (++ia == GDR) {
          ia = 0;
          if (++ib == GDC) {
            ib = 0;
            ++ic;
          }
        }
      }
    }
    // Store X_q (already scaled by 1/N_h), conjugated for the inverse pass,
    // at the stored member, and conj at the partner's stored -k.
    // Branch-free: a store with no target goes to the spare entry lds[S*T].
    auto emit = [&](int q, float2 xs) {
      const bool direct = li[q] >= 0;
      const int a1 = direct ? li[q] : (g.selfc ? S * T : -1 - li[q]);
      lds[a1] = direct ? make_float2(xs.x, -xs.y) : xs;
      lds[mi[q] >= 0 ? mi[q] : S * T] = xs;
    };
    float2 mean;  // (1/d) sum_b L_b X_b of the new x, for the data residual
    if (!a.a_pos && g.js == 0 && g.jn == 0 && g.jm == 0) {
      // Zero-frequency group: member 0 is k = 0 with A = 0. Exact elimination
      // of (1/d) conj(L) L^T X + diag(A) X = B, in FP64.
      float2 L0 = lcur[0], B0 = B[0];
      if (LANES > 1) {
        L0 = make_float2(__shfl(L0.x, gbase), __shfl(L0.y, gbase));
        B0 = make_float2(__shfl(B0.x, gbase), __shfl(B0.y, gbase));
      }
      const double l0r = L0.x, l0i = L0.y;
      const double l0n = l0r * l0r + l0i * l0i;
      if (l0n == 0.0) {
        a.ctrl->status = SR3D_ERR_SINGULAR;
        a.ctrl->done = 1;
#pragma unroll
        for (int q = 0; q < DL; ++q)
          if (EXACT || m0 + q < D) emit(q, make_float2(0.f, 0.f));
        mean = make_float2(0.f, 0.f);
      } else {
        const double br = B0.x, bi = B0.y;
        // s = sum_b L_b X_b = d B_0 / conj(L_0)
        const double sr = (double)D * (br * l0r - bi * l0i) / l0n;
        const double si = (double)D * (br * l0i + bi * l0r) / l0n;
        double accr = 0.0, acci = 0.0;
#pragma unroll
        for (int q = 0; q < DL; ++q) {
          if ((m0 + q > 0) && (EXACT || m0 + q < D)) {
            const double lr = lcur[q].x, lq = lcur[q].y;
            const double tr = (lr * sr + lq * si) / (double)D;
            const double ti = (lr * si - lq * sr) / (double)D;
            const double xr = ((double)B[q].x - tr) / (double)A[q];
            const double xi = ((double)B[q].y - ti) / (double)A[q];
            emit(q, make_float2((float)xr * a.scale, (float)xi * a.scale));
            accr += lr * xr - lq * xi;
            acci += lr * xi + lq * xr;
          }
        }
        if (LANES > 1) {  // lane totals in lane order
          double tr = 0.0, ti = 0.0;
#pragma unroll
          for (int j = 0; j < LANES; ++j) {
            tr += __shfl(accr, gbase + j);
            ti += __shfl(acci, gbase + j);
          }
          accr = tr;
          acci = ti;
        }
        const double nr = sr - accr, ni = si - acci;
        if (sub == 0)
          emit(0, make_float2((float)((nr * l0r + ni * l0i) / l0n) * a.scale,
                              (float)((ni * l0r - nr * l0i) / l0n) * a.scale));
        mean = make_float2((float)(sr / (double)D), (float)(si / (double)D));
      }
    } else {
      // Leave-one-out Woodbury solve in FP32 (the unfused fold kernel's
      // formula, with hardware reciprocals):
      //   X_a = [B_a (d + S_a^(-a)) - conj(L_a) S_b^(-a)] / [A_a (d + S_a)],
      //   S_a = sum_b |L_b|^2 / A_b,  S_b = sum_b L_b B_b / A_b.
      // The leave-one-out sums are prefix + suffix sums over the members;
      // across the lanes of a group, each lane adds the totals of the lanes
      // before and after it. The group's mean (1/d) sum_b L_b X_b equals
      // S_b / (d + S_a).
      float inv[DL], pt[DL], preP[DL];
      float2 qt[DL], preQ[DL];
      float sp = 0.f;
      float2 sq = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < DL; ++q) {
        if (EXACT || m0 + q < D) {
          inv[q] = __builtin_amdgcn_rcpf(A[q]);
          const float2 l = lcur[q];
          const float2 lb = s_mul(l, B[q]);
          pt[q] = (l.x * l.x + l.y * l.y) * inv[q];
          qt[q] = make_float2(lb.x * inv[q], lb.y * inv[q]);
          preP[q] = sp;
          preQ[q] = sq;
          sp += pt[q];
          sq.x += qt[q].x;
          sq.y += qt[q].y;
        }
      }
      // other lanes' totals: before this lane (pP, pQ), after it (fP, fQ), all (tP, tQ)
      float pP = 0.f, fP = 0.f, tP = sp;
      float2 pQ = make_float2(0.f, 0.f), fQ = pQ, tQ = sq;
      if (LANES > 1) {
        tP = 0.f;
        tQ = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < LANES; ++j) {
          const float vP = __shfl(sp, gbase + j);
          const float vx = __shfl(sq.x, gbase + j), vy = __shfl(sq.y, gbase + j);
          tP += vP;
          tQ.x += vx;
          tQ.y += vy;
          if (j < sub) {
            pP += vP;
            pQ.x += vx;
            pQ.y += vy;
          }
        }
#pragma unroll
        for (int j = LANES - 1; j >= 0; --j) {
          const float vP = __shfl(sp, gbase + j);
          const float vx = __shfl(sq.x, gbase + j), vy = __shfl(sq.y, gbase + j);
          if (j > sub) {
            fP += vP;
            fQ.x += vx;
            fQ.y += vy;
          }
        }
      }
      const float rS = __builtin_amdgcn_rcpf(fd + tP);
      const float rSs = rS * a.scale;
      float suP = LANES > 1 ? fP : 0.f;
      float2 suQ = LANES > 1 ? fQ : make_float2(0.f, 0.f);
#pragma unroll
      for (int q = DL - 1; q >= 0; --q) {
        if (EXACT || m0 + q < D) {
          const float2 l = lcur[q];
          const float pre = LANES > 1 ? pP + preP[q] : preP[q];
          const float2 preq = LANES > 1 ? make_float2(pQ.x + preQ[q].x, pQ.y + preQ[q].y) : preQ[q];
          const float saL = pre + suP;
          const float2 sbL = make_float2(preq.x + suQ.x, preq.y + suQ.y);
          const float2 t = s_mul(s_conj(l), sbL);
          const float nd = fd + saL;
          const float rden = inv[q] * rSs;
          emit(q, make_float2((B[q].x * nd - t.x) * rden, (B[q].y * nd - t.y) * rden));
          suP += pt[q];
          suQ.x += qt[q].x;
          suQ.y += qt[q].y;
        }
      }
      mean = make_float2(tQ.x * rS, tQ.y * rS);
    }
    // The LR spectrum of D H x at j and, where it is a stored entry too, at -j.
    if (a.dhx && sub == 0) {
      const int Mlh = a.Ml / 2 + 1;
      gst2(a.dhx, ((uint32_t)(g.js * a.Nl + g.jn) * Mlh + g.jm) * 8u, mean);
      const int jmp = g.jm ? a.Ml - g.jm : 0;
      if (!g.selfc && jmp < Mlh) {
        const int jsp = g.js ? a.Sl - g.js : 0, jnp = g.jn ? a.Nl - g.jn : 0;
        gst2(a.dhx, ((uint32_t)(jsp * a.Nl + jnp) * Mlh + jmp) * 8u, s_conj(mean));
      }
    }
    // Data residual of the new x at j (and, for a pair, at -j); one lane per group.
    if (a.partial && sub == 0) {
      const Acc rr = (Acc)Yj.x - (Acc)mean.x;
      const Acc ri = (Acc)Yj.y - (Acc)mean.y;
      resid += (g.selfc ? (Acc)1 : (Acc)2) * (rr * rr + ri * ri);
    }
  }
  __syncthreads();
  fft_passes<S, T, TP, 0, 1>(lds, stw);
  // The tile indices are recomputed here rather than kept live from the load
  // phase (an empty asm hides that this is the same thread index).
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  if (pairs) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int w2 = tid + k * kThreads;
      const int s = w2 / (T / 2), line = 2 * (w2 - s * (T / 2));
      const int off = (w2 < S * T / 2) ? ut.loff[line] : -1;
      if (off >= 0) {
        const f32x4 v = reinterpret_cast<const f32x4 *>(lds)[w2];
        gst4(a.W, ((uint32_t)s * pl + (uint32_t)off) * 8u, f32x4{v.x, -v.y, v.z, -v.w});
      }
    }
  } else
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int w = tid + k * kThreads;
    const int s = w / T, line = w - s * T;
    const int off = (w < S * T) ? ut.loff[line] : -1;
    if (off >= 0) {
      const float2 v = lds[w];
      gst2(a.W, ((uint32_t)s * pl + (uint32_t)off) * 8u, make_float2(v.x, -v.y));
    }
  }
  if (a.partial) {
    const Acc sum = unit_sum<Acc>(resid, red);
    if (threadIdx.x == 0) reinterpret_cast<Acc *>(a.partial)[u] = sum;
  }
}

// Two workgroups per CU (the LDS tile allows two); every instance holds 8
// members per lane. GR > 0: every volume of the launch has m and n rates GR.
template <int S, int DM, bool EXACT, int GR, typename Acc>
__global__ __launch_bounds__(kThreads, 2) void k_solve_s(const SolveSArgs *__restrict__ descs,
                                                      const int2 *__restrict__ items,
                                                      const float2 *__restrict__ tw) {
  int v = 0, u;
  if (items) {
    const int2 it = items[blockIdx.x];
    v = it.x;
    u = it.y;
  } else {
    u = solve_xcd_unit(blockIdx.x, descs[0].units);
  }
  const SolveSArgs a = descs[v];
  if (a.done && *a.done) return;
  constexpr int T = solve_tile(S);
  __shared__ __align__(16) float2 lds[S * T + 1];  // + a spare entry for stores without a target
  __shared__ float2 stw[S];
  __shared__ float sgs[S];
  __shared__ UnitTabs ut;
  __shared__ Acc red[kThreads / 64];
  solve_s_body<S, DM, EXACT, GR, Acc>(a, u, tw, lds, stw, sgs, ut, red);
}

// The rate the exact instance of member bound DM is specialised for
// (2 x 2 x 2, 2 x 2 x 4 and 4 x 4 x 2).
constexpr int solve_s_fixed_rate(int dm) { return dm == 32 ? 4 : 2; }

template <int S, int DM, typename Acc>
static void launch_solve_s_dm(bool exact, int gr, const SolveSArgs *descs, const int2 *items,
                              int nwg, hipStream_t st) {
  const float2 *tw = twiddles(S);
  constexpr int GRF = solve_s_fixed_rate(DM);
  if (exact && gr == GRF)
    hipLaunchKernelGGL((k_solve_s<S, DM, true, GRF, Acc>), dim3(nwg), dim3(kThreads), 0, st,
                       descs, items, tw);
  else if (exact)
    hipLaunchKernelGGL((k_solve_s<S, DM, true, 0, Acc>), dim3(nwg), dim3(kThreads), 0, st, descs,
                       items, tw);
  else
    hipLaunchKernelGGL((k_solve_s<S, DM, false, 0, Acc>), dim3(nwg), dim3(kThreads), 0, st, descs,
                       items, tw);
}

// dm: member bound of the plan; d: the group size (the instance with
// D = dm fixed at compile time runs when d == dm); gr: the m and n rate
// shared by every volume of the launch, or 0.
template <int S, typename Acc>
static void launch_solve_s_t(int dm, int d, int gr, const SolveSArgs *descs, const int2 *items,
                             int nwg, hipStream_t st) {
  if (dm <= 8) launch_solve_s_dm<S, 8, Acc>(d == 8, gr, descs, items, nwg, st);
  else if (dm <= 16) launch_solve_s_dm<S, 16, Acc>(d == 16, gr, descs, items, nwg, st);
  else launch_solve_s_dm<S, 32, Acc>(d == 32, gr, descs, items, nwg, st);
}

// One launcher per s-length, defined in the instantiating translation units.
#define SR3D_SOLVE_S_LAUNCHER(L)                                                     \
  void solve_s_launch_##L(int dm, int d, int gr, const SolveSArgs *descs,              \
                          const int2 *items, int nwg, bool fp64, hipStream_t st)
#define SR3D_SOLVE_S_DEFINE(L)                                                    \
  SR3D_SOLVE_S_LAUNCHER(L) {                                                      \
    if (fp64) launch_solve_s_t<L, double>(dm, d, gr, descs, items, nwg, st);      \
    else launch_solve_s_t<L, float>(dm, d, gr, descs, items, nwg, st);            \
  }
#define SR3D_SOLVE_S_LENGTHS(X) \
  X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

inline bool solve_s_len(int S) {
  switch (S) {
#define SR3D_CASE(L) case L:
    SR3D_SOLVE_S_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
    return true;
    default:
      return false;
  }
}

#define SR3D_DECL(L) SR3D_SOLVE_S_LAUNCHER(L);
SR3D_SOLVE_S_LENGTHS(SR3D_DECL)
#undef SR3D_DECL

}  // namespace sr3d
