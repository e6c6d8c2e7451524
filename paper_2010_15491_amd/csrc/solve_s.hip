// Fused x-update along s: forward s-FFT, alias-group solve (Algorithm 1 step
// 5a through eq. (8)-(12)) and inverse s-FFT in one pass over the spectrum.
//
// After the m and n passes, the spectrum of Theta is S x N x Mh complex. The
// x-update couples only the d members of an alias group (k = j + (c S_l,
// b N_l, a M_l)), and a member with k_m >= Mh is the conjugate of the stored
// entry at -k. A unit of work (one workgroup) takes the stored (k_n, k_m)
// columns of a set of LR columns closed under negation, so every member and
// every mirror it needs is one of its own s-lines: it loads those lines into
// LDS, transforms them along s, solves the groups, transforms back and writes
// the lines once. The spectrum makes one round trip through HBM instead of
// three.
//
// Groups j and -j have conjugate problems (real PSF, real data), so only one
// of each pair is solved: with j_m the representative of its class
// {j_m, -j_m mod M_l}, and, when the class is self-conjugate, the pair member
// with the smaller (j_s, j_n) index. The solved group writes X_k for its
// stored members and conj(X_k) at the stored -k of the partner group. The
// pointwise formulas are those of the unfused fold kernel (leave-one-out
// Woodbury in FP32, here with hardware reciprocals; exact FP64 elimination of
// the zero-frequency group). Kernel instances live in solve_s_i*.hip.
#include "solve_s_core.h"

namespace sr3d {

// ---------------------------------------------------------------------------
// Host plan
// ---------------------------------------------------------------------------

SolveSPlan solve_s_plan(int S, int N, int M, int dr, int dc, int ds) {
  SolveSPlan P{};
  P.fused = false;
  const int D = dr * dc * ds;
  if (!solve_s_len(S) || D > 32) return P;
  P.dm = D <= 8 ? 8 : D <= 16 ? 16 : 32;
  const int Sl = S / ds, Nl = N / dc, Ml = M / dr, Mh = M / 2 + 1;
  const int T = solve_tile(S);
  // m classes {j, -j mod M_l}, representative j <= M_l - j; each holds the
  // stored k_m (< Mh) congruent to j or -j, in increasing k_m.
  const int NC = Ml / 2 + 1;
  std::vector<std::vector<int>> cls(NC);
  for (int k = 0; k < Mh; ++k) {
    int j = k % Ml;
    if (Ml - j < j) j = Ml - j;
    cls[j].push_back(k);
  }
  int csize = 1;
  for (auto &c : cls) csize = (int)c.size() > csize ? (int)c.size() : csize;
  // n-groups: {0, N_l/2} (both self-conjugate) for even N_l, {0} for odd,
  // then {g, N_l - g}.
  std::vector<int> nj;
  if (Nl % 2 == 0) {
    nj.push_back(0);
    nj.push_back(Nl / 2);
    for (int gg = 1; gg < Nl / 2; ++gg) {
      nj.push_back(gg);
      nj.push_back(Nl - gg);
    }
  } else {
    nj.push_back(0);
    nj.push_back(-1);
    for (int gg = 1; 2 * gg < Nl; ++gg) {
      nj.push_back(gg);
      nj.push_back(Nl - gg);
    }
  }
  const int NG = (int)nj.size() / 2;
  const int rows_max = (nj[1] >= 0 || NG > 1) ? 2 * dc : dc;
  const int KM = T / rows_max;  // stored m columns per unit
  if (KM < csize) return P;
  // m-blocks: consecutive classes, greedily, while the columns fit.
  std::vector<int> bstart;
  int cols = KM + 1;
  for (int j = 0; j < NC; ++j) {
    const int sz = (int)cls[j].size();
    if (cols + sz > KM) {
      bstart.push_back(j);
      cols = 0;
    }
    cols += sz;
  }
  const int NB = (int)bstart.size();
  bstart.push_back(NC);
  int CB = 1;
  for (int b = 0; b < NB; ++b) CB = bstart[b + 1] - bstart[b] > CB ? bstart[b + 1] - bstart[b] : CB;
  if (CB * dr > 64) return P;
  P.NG = NG;
  P.NB = NB;
  P.CB = CB;
  P.units = NG * NB;
  P.gmax = Sl * 2 * CB;
  P.o_p0 = 2 * Mh;
  P.o_cnt = P.o_p0 + NB;
  P.o_mj = P.o_cnt + NB;
  P.o_nj = P.o_mj + NB * CB;
  P.tab.assign((size_t)P.o_nj + 2 * NG, -1);
  int pos = 0;
  for (int b = 0; b < NB; ++b) {
    P.tab[P.o_p0 + b] = pos;
    int cnt = 0;
    for (int j = bstart[b]; j < bstart[b + 1]; ++j) {
      P.tab[P.o_mj + b * CB + (j - bstart[b])] = j;
      for (int k : cls[j]) {
        P.tab[pos] = k;       // kofp
        P.tab[Mh + k] = pos;  // posk
        ++pos;
        ++cnt;
      }
    }
    P.tab[P.o_cnt + b] = cnt;
  }
  for (int i = 0; i < 2 * NG; ++i) P.tab[P.o_nj + i] = nj[i];
  // Long rows are padded to a multiple of 16 complex values (128 bytes), so
  // row starts and the n-pass tiles are cache-line aligned.
  P.pitch = Mh >= 64 ? (Mh + 15) / 16 * 16 : Mh;
  P.fused = true;
  return P;
}

// Setup: Lambda of every member (conjugated where the member is a mirror) and
// the LR spectrum Y_j of every solved group, in (unit, member, slot) order.
__global__ __launch_bounds__(kThreads) void k_solve_s_gather(SolveSArgs a,
                                                             const float2 *__restrict__ lam,
                                                             const float2 *__restrict__ yh,
                                                             int Mlh, float2 *Lg, float2 *Yg) {
  const long i = (long)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (long)a.units * a.gmax) return;
  const int u = (int)(i / a.gmax), slot = (int)(i - (long)u * a.gmax);
  const int gn = u / a.NB, bm = u - gn * a.NB;
  const int j0 = a.tab[a.o_nj + 2 * gn], j1 = a.tab[a.o_nj + 2 * gn + 1];
  SlotGroup g;
  const int *mj = a.tab + a.o_mj + bm * a.CB;
  const int nc = block_classes(mj, a.CB);
  if (slot >= a.Sl * 2 * nc || !slot_group(a, mj, nc, j0, j1, slot, g)) {
    Yg[i] = make_float2(0.f, 0.f);
    if (lam)
      for (int q = 0; q < a.D; ++q) Lg[((long)u * a.D + q) * a.gmax + slot] = make_float2(0.f, 0.f);
    return;
  }
  float2 Yj;
  if (g.jm < Mlh) {
    Yj = yh[((long)g.js * a.Nl + g.jn) * Mlh + g.jm];
  } else {
    const int ms = (a.Sl - g.js) % a.Sl, mn = (a.Nl - g.jn) % a.Nl;
    Yj = s_conj(yh[((long)ms * a.Nl + mn) * Mlh + (a.Ml - g.jm)]);
  }
  Yg[i] = Yj;
  if (!lam) return;  // Y alone
  int ia = 0, ib = 0, ic = 0;
  for (int q = 0; q < a.D; ++q) {
    const int km = g.jm + ia * a.Ml, kn = g.jn + ib * a.Nl, ks = g.js + ic * a.Sl;
    float2 l;
    if (km < a.Mh) {
      l = lam[((long)ks * a.N + kn) * a.Mh + km];
    } else {
      const int ms = (a.S - ks) % a.S, mn = (a.N - kn) % a.N;
      l = s_conj(lam[((long)ms * a.N + mn) * a.Mh + (a.M - km)]);
    }
    Lg[((long)u * a.D + q) * a.gmax + slot] = l;
    if (++ia == a.dr) {
      ia = 0;
      if (++ib == a.dc) {
        ib = 0;
        ++ic;
      }
    }
  }
}

hipError_t solve_s(int S, int dm, int d, int gr, const SolveSArgs *descs, const int2 *items,
                   int nwg, bool fp64, hipStream_t st) {
  if (nwg == 0) return hipSuccess;
  if (!twiddles(S)) return hipErrorInvalidValue;
  switch (S) {
#define SR3D_CASE(L)                                        \
  case L:                                                   \
    solve_s_launch_##L(dm, d, gr, descs, items, nwg, fp64, st); \
    break;
    SR3D_SOLVE_S_LENGTHS(SR3D_CASE)
#undef SR3D_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t solve_s_gather(const SolveSArgs &a, const float2 *lam, const float2 *yh, int Mlh,
                          hipStream_t st) {
  const long n = (long)a.units * a.gmax;
  hipLaunchKernelGGL(k_solve_s_gather, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, a, lam, yh, Mlh, const_cast<float2 *>(a.Lg),
                     const_cast<float2 *>(a.Yg));
  return hipGetLastError();
}

hipError_t solve_s_gather_y(const SolveSArgs &a, const float2 *yh, int Mlh, hipStream_t st) {
  return solve_s_gather(a, nullptr, yh, Mlh, st);
}

}  // namespace sr3d
