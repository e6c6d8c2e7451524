// Multi-frame fold / solve / unfold (3D multi-frame SR, which the paper's
// conclusion names as future work). F LR frames y_f = D S_f H x + n_f of one
// HR volume, S_f a circular shift by t_f HR voxels ((S_f z)[i] = z[i + t_f]).
// With F(S_f z)_k = w_f(k) Z_k, w_f(k) = exp(2 pi i k . t_f / n), eq. (8)
// turns the normal equations of eq. (6) (and of Algorithm 1 step 5a) into one
// d x d system per alias group j with one rank-one term per frame:
//   (1/d) sum_f conj(v_f) v_f^T X + diag(A) X = B,   v_f,a = w_f(k_a) Lambda_a,
//   B_a = sum_f conj(v_f,a) Y_f,j + c W_a.
// Woodbury with the F x F matrix Q = d I + V^T A^-1 conj(V) gives
//   Q t = V^T A^-1 B,   X_a = (B_a - sum_f conj(v_f,a) t_f) / A_a,
// solved in FP64 (complex Cholesky) by the lanes that own the group. In a
// TV solve the zero-frequency member has A = 0; that group is solved by the
// Schur complement of member 0, with the same Woodbury solve for the rest.
// The phase of member k = (j_m + a M_l, j_n + b N_l, j_s + c S_l) splits into
// a per-group factor exp(2 pi i (j_m t_m / M + j_n t_n / N + j_s t_s / S))
// (from the FFT twiddle tables, w = conj(tw_n[k t mod n])) and a per-member
// root of unity exp(2 pi i (a t_m / d_r + b t_n / d_c + c t_s / d_s)), the
// same for every group (a host table).
#include "sr3d_internal.h"

namespace sr3d {

namespace {

struct zd {
  double x, y;
};
__device__ __forceinline__ zd zmul(zd a, zd b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ zd zconj(zd a) { return {a.x, -a.y}; }
__device__ __forceinline__ zd zadd(zd a, zd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ zd zsub(zd a, zd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ zd zscale(zd a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ zd zf(float2 a) { return {(double)a.x, (double)a.y}; }

// exp(+2 pi i k t / n) from the table tw[k] = exp(-2 pi i k / n)
// (0 <= k < n <= 1024, |t| < 2^20, so k t fits 32 bits).
__device__ __forceinline__ float2 phase(const float2 *tw, int n, int k, int t) {
  int kt = (k * t) % n;
  kt += kt < 0 ? n : 0;
  const float2 w = tw[kt];
  return make_float2(w.x, -w.y);
}
__device__ __forceinline__ float2 fmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Solves Q z = b for the Hermitian positive definite FM x FM matrix Q (upper
// triangle used) by a complex Cholesky factorisation Q = R^H R, in place.
// Frames beyond the call's F enter as rows d e_f with b_f = 0 (solution 0),
// so the loops run over all FM and unroll.
template <int FM>
__device__ __forceinline__ void chol_solve(zd (&Q)[FM][FM], zd (&b)[FM]) {
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double di = Q[i][i].x;
#pragma unroll
    for (int k = 0; k < i; ++k) di -= Q[k][i].x * Q[k][i].x + Q[k][i].y * Q[k][i].y;
    const double rii = sqrt(fmax(di, 0.0));
    const double inv = rii > 0.0 ? 1.0 / rii : 0.0;
    Q[i][i] = {rii, inv};  // keep 1/R_ii in the imaginary slot
#pragma unroll
    for (int j = i + 1; j < FM; ++j) {
      zd s = Q[i][j];
#pragma unroll
      for (int k = 0; k < i; ++k) s = zsub(s, zmul(zconj(Q[k][i]), Q[k][j]));
      Q[i][j] = zscale(s, inv);
    }
  }
  // R^H y = b
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    zd s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = zsub(s, zmul(zconj(Q[k][i]), b[k]));
    b[i] = zscale(s, Q[i][i].y);
  }
  // R z = y
#pragma unroll
  for (int i = FM - 1; i >= 0; --i) {
    zd s = b[i];
#pragma unroll
    for (int k = i + 1; k < FM; ++k) s = zsub(s, zmul(Q[i][k], b[k]));
    b[i] = zscale(s, Q[i][i].y);
  }
}

// Sums over the LANES consecutive lanes of a group (xor butterfly: the same
// bits in every lane of the group).
template <int LANES>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int o = 1; o < LANES; o <<= 1) v += __shfl_xor(v, o);
  return v;
}
template <int LANES>
__device__ __forceinline__ zd gsum(zd v) {
  return {gsum<LANES>(v.x), gsum<LANES>(v.y)};
}

// One thread per group up to d = 8. The 16- and 32-member groups are spread
// over LANES = d / 4 consecutive lanes, 4 members each (lane sub holds
// members 4 sub .. 4 sub + 3): the F x F system and its right-hand side are
// sums over members, reduced across the group's lanes, and every lane
// factorises the same reduced matrix. (Splitting the 8-member groups as well
// measured slower: each lane repeats the FP64 factorisation.) A workgroup
// handles kThreads groups in LANES passes, so the partial sums stay one per
// workgroup of kThreads groups.
template <int D, int FM, typename Acc>
__global__ __launch_bounds__(kThreads) void k_fold_solve_mf(MfArgs a) {
  if (a.done && *a.done) return;
  constexpr int DL = D <= 8 ? D : 4, LANES = D / DL, GPP = kThreads / LANES;
  __shared__ Acc sh[kThreads / 64];
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  const int F = a.F;
  const int sub = (int)threadIdx.x % LANES;
  const int lbase = ((int)threadIdx.x & 63) - sub;  // lane of the group's first member
  Acc resid = 0;
  for (int pass = 0; pass < LANES; ++pass) {
    const long g = (long)blockIdx.x * kThreads + pass * GPP + (long)threadIdx.x / LANES;
    if (g >= ngroups) continue;  // the same for every lane of the group
    const int jm = (int)(g % a.ml_eff);
    const long r1 = g / a.ml_eff;
    const int jn = (int)(r1 % a.Nl);
    const int js = (int)(r1 / a.Nl);
    // LR spectra of the frames at j (stored half, mirrored otherwise)
    zd Y[FM];
    {
      long id;
      bool mir = false;
      if (jm < a.Mlh) {
        id = ((long)js * a.Nl + jn) * a.Mlh + jm;
      } else {
        id = ((long)((a.Sl - js) % a.Sl) * a.Nl + (a.Nl - jn) % a.Nl) * a.Mlh + (a.Ml - jm);
        mir = true;
      }
#pragma unroll
      for (int f = 0; f < FM; ++f) {
        Y[f] = {0.0, 0.0};
        if (f < F) {
          const float2 y = a.Yf[(long)f * a.nlspec + id];
          Y[f] = {(double)y.x, mir ? -(double)y.y : (double)y.y};
        }
      }
    }
    // per-group phase factor of each frame
    float2 base[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f)
      base[f] = f < F ? fmul(fmul(phase(a.twm, a.M, jm, a.t[f][0]), phase(a.twn, a.N, jn, a.t[f][1])),
                             phase(a.tws, a.S, js, a.t[f][2]))
                      : make_float2(0.f, 0.f);
    // this lane's members q = sub DL + i
    const int q0l = sub * DL;
    zd lam[DL], B[DL];
    double A[DL];
    long idx[DL];
    bool own[DL];
    int ia = q0l % a.dr, ib = (q0l / a.dr) % a.dc, ic = q0l / (a.dr * a.dc);
#pragma unroll
    for (int i = 0; i < DL; ++i) {
      const int q = q0l + i;
      const int km = jm + ia * a.Ml, kn = jn + ib * a.Nl, ks = js + ic * a.Sl;
      const bool direct = km < a.Mh;
      long id;
      if (direct) id = ((long)ks * a.N + kn) * a.Mh + km;
      else id = ((long)((a.S - ks) % a.S) * a.N + (a.N - kn) % a.N) * a.Mh + (a.M - km);
      float2 l = a.Lam[id];
      float2 w = a.W ? a.W[id] : make_float2(0.f, 0.f);
      if (!direct) {
        l.y = -l.y;
        w.y = -w.y;
      }
      lam[i] = zf(l);
      A[i] = a.tv ? (double)a.coefA * ((double)a.gs[ks] + (double)a.gn[kn] + (double)a.gm[km])
                  : (double)a.coefA;
      zd b = zscale(zf(w), (double)a.cw);
#pragma unroll
      for (int f = 0; f < FM; ++f) {
        if (f < F) {
          const float2 ph = fmul(base[f], a.r[f][q]);
          b = zadd(b, zmul(zconj(zmul(zf(ph), lam[i])), Y[f]));
        }
      }
      B[i] = b;
      idx[i] = id;
      own[i] = direct;
      if (++ia == a.dr) {
        ia = 0;
        if (++ib == a.dc) {
          ib = 0;
          ++ic;
        }
      }
    }
    auto v_of = [&](int f, int i) { return zmul(zf(fmul(base[f], a.r[f][q0l + i])), lam[i]); };
    // Woodbury over the members q >= qs (A > 0 there): Q t = V^T A^-1 z.
    auto woodbury = [&](int qs, const zd *z, zd *out) {
      zd Q[FM][FM], t[FM];
#pragma unroll
      for (int f = 0; f < FM; ++f) {
        t[f] = {0.0, 0.0};
#pragma unroll
        for (int h = 0; h < FM; ++h) Q[f][h] = {(LANES == 1 && f == h) ? (double)D : 0.0, 0.0};
      }
#pragma unroll
      for (int i = 0; i < DL; ++i) {
        if (q0l + i < qs) continue;
        const double ia_ = 1.0 / A[i];
        zd v[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) v[f] = f < F ? v_of(f, i) : zd{0.0, 0.0};
#pragma unroll
        for (int f = 0; f < FM; ++f) {
          t[f] = zadd(t[f], zscale(zmul(v[f], z[i]), ia_));
#pragma unroll
          for (int h = f; h < FM; ++h) Q[f][h] = zadd(Q[f][h], zscale(zmul(v[f], zconj(v[h])), ia_));
        }
      }
      if (LANES > 1) {
#pragma unroll
        for (int f = 0; f < FM; ++f) {
          t[f] = gsum<LANES>(t[f]);
#pragma unroll
          for (int h = f; h < FM; ++h) Q[f][h] = gsum<LANES>(Q[f][h]);
          Q[f][f].x += (double)D;
        }
      }
      chol_solve<FM>(Q, t);
#pragma unroll
      for (int i = 0; i < DL; ++i) {
        if (q0l + i < qs) continue;
        zd s = z[i];
#pragma unroll
        for (int f = 0; f < FM; ++f)
          if (f < F) s = zsub(s, zmul(zconj(v_of(f, i)), t[f]));
        out[i] = zscale(s, 1.0 / A[i]);
      }
    };
    zd X[DL];
    if (a.tv && g == 0) {
      // Zero-frequency group: member 0 (lane 0 of the group) has A = 0. Schur
      // complement of member 0 with K_rr = diag(A_r) + (1/d) conj(V_r) V_r^T
      // (Woodbury):
      //   X_0 = (B_0 - K_0r K_rr^-1 B_r) / (k_00 - K_0r K_rr^-1 K_r0),
      //   X_r = K_rr^-1 (B_r - K_r0 X_0).
      zd lam0 = lam[0], B0 = B[0];
      if (LANES > 1) {
        lam0 = {__shfl(lam0.x, lbase), __shfl(lam0.y, lbase)};
        B0 = {__shfl(B0.x, lbase), __shfl(B0.y, lbase)};
      }
      zd kr0[DL], u1[DL], u2[DL];
      double k00 = 0.0;
#pragma unroll
      for (int i = 0; i < DL; ++i) kr0[i] = u1[i] = u2[i] = {0.0, 0.0};
#pragma unroll
      for (int f = 0; f < FM; ++f) {
        if (f >= F) continue;
        const zd v0 = zmul(zf(fmul(base[f], a.r[f][0])), lam0);
        k00 += (v0.x * v0.x + v0.y * v0.y) / (double)D;
#pragma unroll
        for (int i = 0; i < DL; ++i)
          if (q0l + i >= 1) kr0[i] = zadd(kr0[i], zscale(zmul(zconj(v_of(f, i)), v0), 1.0 / D));
      }
      woodbury(1, B, u1);    // K_rr^-1 B_r
      woodbury(1, kr0, u2);  // K_rr^-1 K_r0
      zd num = {0.0, 0.0}, den = {0.0, 0.0};
#pragma unroll
      for (int i = 0; i < DL; ++i) {
        if (q0l + i < 1) continue;
        // K_0r = conj(K_r0)^T (K is Hermitian)
        num = zadd(num, zmul(zconj(kr0[i]), u1[i]));
        den = zadd(den, zmul(zconj(kr0[i]), u2[i]));
      }
      num = zsub(B0, gsum<LANES>(num));
      den = zsub(zd{k00, 0.0}, gsum<LANES>(den));
      const double dn = den.x * den.x + den.y * den.y;
      if (!(dn > 0.0)) {
        a.ctrl->status = SR3D_ERR_SINGULAR;
        a.ctrl->done = 1;
#pragma unroll
        for (int i = 0; i < DL; ++i) X[i] = {0.0, 0.0};
      } else {
        const zd x0 = zscale(zmul(num, zconj(den)), 1.0 / dn);
        zd z[DL];
#pragma unroll
        for (int i = 0; i < DL; ++i) z[i] = zsub(B[i], zmul(kr0[i], x0));
        woodbury(1, z, X);
        if (sub == 0) X[0] = x0;
      }
    } else {
      woodbury(0, B, X);
    }
    // Data residual of the new x: sum_f |Y_f,j - (1/d) sum_a v_f,a X_a|^2.
    if (a.partial) {
      Acc wgt = 1;
      if (a.ml_eff < a.Ml && jm != 0 && 2 * jm != a.Ml) wgt = 2;
#pragma unroll
      for (int f = 0; f < FM; ++f) {
        if (f >= F) continue;
        zd m = {0.0, 0.0};
#pragma unroll
        for (int i = 0; i < DL; ++i) m = zadd(m, zmul(v_of(f, i), X[i]));
        m = gsum<LANES>(m);
        const zd r = zsub(Y[f], zscale(m, 1.0 / D));
        if (sub == 0) resid += wgt * (Acc)(r.x * r.x + r.y * r.y);
      }
    }
#pragma unroll
    for (int i = 0; i < DL; ++i)
      if (own[i]) a.X[idx[i]] = make_float2((float)(X[i].x * a.scale), (float)(X[i].y * a.scale));
  }
  if (a.partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) resid += __shfl_xor(resid, off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = resid;
    __syncthreads();
    if (threadIdx.x == 0) {
      Acc s = 0;
      for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
      reinterpret_cast<Acc *>(a.partial)[blockIdx.x] = s;
    }
  }
}

template <int FM, typename Acc>
hipError_t launch_mf(const MfArgs &a, hipStream_t st) {
  const int D = a.dr * a.dc * a.ds;
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  dim3 g((unsigned)((ngroups + kThreads - 1) / kThreads)), b(kThreads);
  switch (D) {
#define SR3D_D(DD)                                                        \
  case DD:                                                                \
    hipLaunchKernelGGL((k_fold_solve_mf<DD, FM, Acc>), g, b, 0, st, a);   \
    break;
    SR3D_D(1) SR3D_D(2) SR3D_D(4) SR3D_D(8) SR3D_D(16) SR3D_D(32)
#undef SR3D_D
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool fold_mf_supported(int d, int nframes) {
  return (d == 1 || d == 2 || d == 4 || d == 8 || d == 16 || d == 32) && nframes >= 1 &&
         nframes <= kMaxFrames;
}

int fold_mf_blocks(const MfArgs &a) {
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  return (int)((ngroups + kThreads - 1) / kThreads);
}

hipError_t fold_solve_mf(const MfArgs &a, bool fp64, hipStream_t st) {
  if (!fold_mf_supported(a.dr * a.dc * a.ds, a.F)) return hipErrorInvalidValue;
  prof_begin(kStFold, st);
  hipError_t e;
  if (a.F <= 2) e = fp64 ? launch_mf<2, double>(a, st) : launch_mf<2, float>(a, st);
  else e = fp64 ? launch_mf<kMaxFrames, double>(a, st) : launch_mf<kMaxFrames, float>(a, st);
  prof_end(st);
  return e;
}

}  // namespace sr3d
