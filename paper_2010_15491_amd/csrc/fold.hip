// Fold / solve / unfold: the pointwise part of eq. (12) and Algorithm 1 step 5a.
//
// By eq. (8), F D^H D F^H replaces every member of an alias group by the group
// mean, so the normal equations of the x-update decouple into one small
// system per LR frequency j (Sec. III-A, the definition of underline-Lambda):
//   conj(L_a) (1/d) sum_b L_b X_b + A_a X_a = B_a ,  a = 1..d,
// with A = 2 lambda (Tikhonov) or A = mu G (TV, G = |Sigma_h|^2+|Sigma_v|^2+
// |Sigma_s|^2), and B = conj(L) F D^H y + c W, where F D^H y is the LR
// spectrum of y replicated over the group and W = F xbar or F Theta.
// Eq. (12) (Woodbury) solves it as
//   X_a = [B_a (d + S_a) - conj(L_a) S_b] / [A_a (d + S_a)],
//   S_a = sum_b |L_b|^2 / A_b, S_b = sum_b L_b B_b / A_b .
// In FP32 the two terms of the numerator nearly cancel; substituting
// S = S^(-a) + (own term) removes the cancellation exactly:
//   X_a = [B_a (d + S_a^(-a)) - conj(L_a) S_b^(-a)] / [A_a (d + S_a)],
// with the leave-one-out sums S^(-a) built from prefix and suffix sums.
// The group holding k = 0 in a TV solve has A = 0 at k = 0 (Gamma = 1/G is
// unbounded there, Algorithm 1 step 4); it is solved by exact elimination in
// FP64 by the one thread that owns it.
//
// Half-spectrum storage: member k with k_m <= M/2 is stored at k; otherwise
// its value is conj of the entry at -k. One thread per group j reads all d
// members and writes only the members it stores, so every stored entry is
// written exactly once (by the group k mod LR).
#include "sr3d_internal.h"

namespace sr3d {

struct cplx {
  float x, y;
};

__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }

template <typename T>
__device__ __forceinline__ T block_reduce_sum(T v, T *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  }
  return r;
}

template <int D, typename Acc>
__device__ __forceinline__ void fold_body(const FoldArgs &a, int bid) {
  __shared__ Acc sh[kThreads / 64];
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  const long g = (long)bid * kThreads + threadIdx.x;
  Acc resid = 0;
  if (g < ngroups) {
    const int jm = (int)(g % a.ml_eff);
    const long r1 = g / a.ml_eff;
    const int jn = (int)(r1 % a.Nl);
    const int js = (int)(r1 / a.Nl);
    // LR spectrum of y at j (stored half, mirrored otherwise)
    float2 Yj;
    if (jm < a.Mlh) {
      Yj = a.Yh[((long)js * a.Nl + jn) * a.Mlh + jm];
    } else {
      const int ms = (a.Sl - js) % a.Sl, mn = (a.Nl - jn) % a.Nl;
      Yj = c_conj(a.Yh[((long)ms * a.Nl + mn) * a.Mlh + (a.Ml - jm)]);
    }
    const float fd = (float)D;
    float2 lam[D], B[D];
    float A[D];
    long idx[D];
    bool own[D];
    int ia = 0, ib = 0, ic = 0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const int km = jm + ia * a.Ml, kn = jn + ib * a.Nl, ks = js + ic * a.Sl;
      const bool direct = km < a.Mh;
      long id;
      if (direct) {
        id = ((long)ks * a.N + kn) * a.Mh + km;
      } else {
        const int ms = (a.S - ks) % a.S, mn = (a.N - kn) % a.N;
        id = ((long)ms * a.N + mn) * a.Mh + (a.M - km);
      }
      float2 l = a.Lam[id];
      float2 w = a.W ? a.W[id] : make_float2(0.f, 0.f);
      if (!direct) {
        l.y = -l.y;
        w.y = -w.y;
      }
      const float Aq = a.tv ? a.coefA * (a.gs[ks] + a.gn[kn] + a.gm[km]) : a.coefA;
      const float2 cb = c_mul(c_conj(l), Yj);
      lam[q] = l;
      B[q] = make_float2(cb.x + a.cw * w.x, cb.y + a.cw * w.y);
      A[q] = Aq;
      idx[q] = id;
      own[q] = direct;
      if (++ia == a.dr) {
        ia = 0;
        if (++ib == a.dc) {
          ib = 0;
          ++ic;
        }
      }
    }
    float2 X[D];
    if (a.tv && g == 0) {
      // Zero-frequency group: member 0 is k = 0 with A = 0. Exact elimination
      // of (1/d) conj(L) L^T X + diag(A) X = B, in FP64.
      const double l0r = lam[0].x, l0i = lam[0].y;
      const double l0n = l0r * l0r + l0i * l0i;
      if (l0n == 0.0) {
        a.ctrl->status = SR3D_ERR_SINGULAR;
        a.ctrl->done = 1;
#pragma unroll
        for (int q = 0; q < D; ++q) X[q] = make_float2(0.f, 0.f);
      } else {
        // s = d B_0 / conj(L_0)  (= sum_b L_b X_b)
        const double br = B[0].x, bi = B[0].y;
        // B0 / conj(L0) = B0 * L0 / |L0|^2
        const double sr = (double)D * (br * l0r - bi * l0i) / l0n;
        const double si = (double)D * (br * l0i + bi * l0r) / l0n;
        double accr = 0.0, acci = 0.0;
#pragma unroll
        for (int q = 1; q < D; ++q) {
          const double lr = lam[q].x, li = lam[q].y;
          // X_q = (B_q - conj(L_q) s / d) / A_q
          const double tr = (lr * sr + li * si) / (double)D;
          const double ti = (lr * si - li * sr) / (double)D;
          const double xr = ((double)B[q].x - tr) / (double)A[q];
          const double xi = ((double)B[q].y - ti) / (double)A[q];
          X[q] = make_float2((float)xr, (float)xi);
          accr += lr * xr - li * xi;
          acci += lr * xi + li * xr;
        }
        // X_0 = (s - sum_{q>0} L_q X_q) / L_0
        const double nr = sr - accr, ni = si - acci;
        X[0] = make_float2((float)((nr * l0r + ni * l0i) / l0n), (float)((ni * l0r - nr * l0i) / l0n));
      }
    } else {
      // Leave-one-out Woodbury solve in FP32.
      float preP[D];
      float2 preQ[D];
      float sp = 0.f;
      float2 sq = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < D; ++q) {
        preP[q] = sp;
        preQ[q] = sq;
        const float inv = 1.0f / A[q];
        sp += (lam[q].x * lam[q].x + lam[q].y * lam[q].y) * inv;
        const float2 lb = c_mul(lam[q], B[q]);
        sq.x += lb.x * inv;
        sq.y += lb.y * inv;
      }
      const float Sa = sp;
      float suP = 0.f;
      float2 suQ = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = D - 1; q >= 0; --q) {
        const float saL = preP[q] + suP;
        const float2 sbL = make_float2(preQ[q].x + suQ.x, preQ[q].y + suQ.y);
        const float2 t = c_mul(c_conj(lam[q]), sbL);
        const float nd = fd + saL;
        const float den = A[q] * (fd + Sa);
        X[q] = make_float2((B[q].x * nd - t.x) / den, (B[q].y * nd - t.y) / den);
        const float inv = 1.0f / A[q];
        suP += (lam[q].x * lam[q].x + lam[q].y * lam[q].y) * inv;
        const float2 lb = c_mul(lam[q], B[q]);
        suQ.x += lb.x * inv;
        suQ.y += lb.y * inv;
      }
    }
    // (1/d) sum_a L_a X_a is the LR spectrum of D H x at j (eq. (8)): the
    // data residual Y_j - it (LR Parseval), and with `dhx` that spectrum at
    // the stored LR entries.
    float2 acc = make_float2(0.f, 0.f);
    if (a.partial || a.dhx) {
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const float2 lx = c_mul(lam[q], X[q]);
        acc.x += lx.x;
        acc.y += lx.y;
      }
    }
    if (a.dhx && jm < a.Mlh)
      a.dhx[((long)js * a.Nl + jn) * a.Mlh + jm] = make_float2(acc.x / fd, acc.y / fd);
    if (a.partial) {
      const Acc rr = (Acc)Yj.x - (Acc)acc.x / (Acc)D;
      const Acc ri = (Acc)Yj.y - (Acc)acc.y / (Acc)D;
      // weight 2 for groups whose conjugate partner is not processed (dr = 1)
      Acc wgt = 1;
      if (a.ml_eff < a.Ml && jm != 0 && 2 * jm != a.Ml) wgt = 2;
      resid = wgt * (rr * rr + ri * ri);
    }
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if (own[q]) a.X[idx[q]] = make_float2(X[q].x * a.scale, X[q].y * a.scale);
    }
  }
  if (a.partial) {
    const Acc s = block_reduce_sum<Acc>(resid, sh);
    if (threadIdx.x == 0) reinterpret_cast<Acc *>(a.partial)[bid] = s;
  }
}

template <int D, typename Acc>
__global__ __launch_bounds__(kThreads) void k_fold_solve(FoldArgs a) {
  if (a.done && *a.done) return;
  fold_body<D, Acc>(a, blockIdx.x);
}

template <int D, typename Acc>
__global__ __launch_bounds__(kThreads) void k_fold_solve_batch(const FoldArgs *__restrict__ descs,
                                                               const int2 *__restrict__ items) {
  const int2 it = items[blockIdx.x];
  const FoldArgs a = descs[it.x];
  if (a.done && *a.done) return;
  fold_body<D, Acc>(a, it.y);
}

int fold_blocks(const FoldArgs &a) {
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  return (int)((ngroups + kThreads - 1) / kThreads);
}

template <typename Acc>
static hipError_t launch_fold(const FoldArgs &a, hipStream_t st) {
  const int D = a.dr * a.dc * a.ds;
  dim3 g((unsigned)fold_blocks(a)), b(kThreads);
  switch (D) {
#define SR3D_D(DD)                                                    \
  case DD:                                                            \
    hipLaunchKernelGGL((k_fold_solve<DD, Acc>), g, b, 0, st, a);      \
    break;
    SR3D_D(1) SR3D_D(2) SR3D_D(3) SR3D_D(4) SR3D_D(6) SR3D_D(8) SR3D_D(9) SR3D_D(12)
    SR3D_D(16) SR3D_D(18) SR3D_D(24) SR3D_D(27) SR3D_D(32) SR3D_D(36) SR3D_D(48) SR3D_D(64)
#undef SR3D_D
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Dual warm start. For x0 with spectrum W, the minimum-norm d solving the
// stationarity of the x-update, mu L^T d = H^T D^T (y - D H x0), is d = L phi
// with phi = (L^T L)^+ H^T D^T (y - D H x0) / mu. In the Fourier domain
//   Phi_k = conj(L_k) Z_j / (mu G_k),  Z_j = Y_j - (1/d) sum_a L_a W_a,
// with Phi_0 = 0. Output scaled by `scale` for the inverse FFT.
template <int D>
__global__ __launch_bounds__(kThreads) void k_dual_init(FoldArgs a) {
  const long ngroups = (long)a.Sl * a.Nl * a.ml_eff;
  const long g = (long)blockIdx.x * kThreads + threadIdx.x;
  if (g >= ngroups) return;
  const int jm = (int)(g % a.ml_eff);
  const long r1 = g / a.ml_eff;
  const int jn = (int)(r1 % a.Nl);
  const int js = (int)(r1 / a.Nl);
  float2 Yj;
  if (jm < a.Mlh) {
    Yj = a.Yh[((long)js * a.Nl + jn) * a.Mlh + jm];
  } else {
    const int ms = (a.Sl - js) % a.Sl, mn = (a.Nl - jn) % a.Nl;
    Yj = c_conj(a.Yh[((long)ms * a.Nl + mn) * a.Mlh + (a.Ml - jm)]);
  }
  float2 lam[D];
  float A[D];
  long idx[D];
  bool own[D];
  float2 z = Yj;
  int ia = 0, ib = 0, ic = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    const int km = jm + ia * a.Ml, kn = jn + ib * a.Nl, ks = js + ic * a.Sl;
    const bool direct = km < a.Mh;
    long id;
    if (direct) {
      id = ((long)ks * a.N + kn) * a.Mh + km;
    } else {
      const int ms = (a.S - ks) % a.S, mn = (a.N - kn) % a.N;
      id = ((long)ms * a.N + mn) * a.Mh + (a.M - km);
    }
    float2 l = a.Lam[id], w = a.W[id];
    if (!direct) {
      l.y = -l.y;
      w.y = -w.y;
    }
    const float2 lw = c_mul(l, w);
    z.x -= lw.x / (float)D;
    z.y -= lw.y / (float)D;
    lam[q] = l;
    A[q] = a.coefA * (a.gs[ks] + a.gn[kn] + a.gm[km]);
    idx[q] = id;
    own[q] = direct;
    if (++ia == a.dr) {
      ia = 0;
      if (++ib == a.dc) {
        ib = 0;
        ++ic;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < D; ++q) {
    if (!own[q]) continue;
    float2 v = make_float2(0.f, 0.f);
    if (A[q] > 0.f) {
      const float2 t = c_mul(c_conj(lam[q]), z);
      v = make_float2(t.x / A[q] * a.scale, t.y / A[q] * a.scale);
    }
    a.X[idx[q]] = v;
  }
}

hipError_t dual_init_spectrum(const FoldArgs &a, hipStream_t st) {
  const int D = a.dr * a.dc * a.ds;
  dim3 g((unsigned)fold_blocks(a)), b(kThreads);
  switch (D) {
#define SR3D_D(DD)                                                 \
  case DD:                                                         \
    hipLaunchKernelGGL((k_dual_init<DD>), g, b, 0, st, a);         \
    break;
    SR3D_D(1) SR3D_D(2) SR3D_D(3) SR3D_D(4) SR3D_D(6) SR3D_D(8) SR3D_D(9) SR3D_D(12)
    SR3D_D(16) SR3D_D(18) SR3D_D(24) SR3D_D(27) SR3D_D(32) SR3D_D(36) SR3D_D(48) SR3D_D(64)
#undef SR3D_D
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Acc>
static hipError_t launch_fold_batch(int D, const FoldArgs *descs, const int2 *items, int nitems,
                                    hipStream_t st) {
  dim3 g((unsigned)nitems), b(kThreads);
  switch (D) {
#define SR3D_D(DD)                                                                 \
  case DD:                                                                         \
    hipLaunchKernelGGL((k_fold_solve_batch<DD, Acc>), g, b, 0, st, descs, items);  \
    break;
    SR3D_D(1) SR3D_D(2) SR3D_D(3) SR3D_D(4) SR3D_D(6) SR3D_D(8) SR3D_D(9) SR3D_D(12)
    SR3D_D(16) SR3D_D(18) SR3D_D(24) SR3D_D(27) SR3D_D(32) SR3D_D(36) SR3D_D(48) SR3D_D(64)
#undef SR3D_D
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t fold_solve_batch(int D, const FoldArgs *descs, const int2 *items, int nitems, bool fp64,
                            hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  return fp64 ? launch_fold_batch<double>(D, descs, items, nitems, st)
              : launch_fold_batch<float>(D, descs, items, nitems, st);
}

hipError_t fold_solve(const FoldArgs &a, bool fp64, hipStream_t st) {
  prof_begin(kStFold, st);
  hipError_t e = fp64 ? launch_fold<double>(a, st) : launch_fold<float>(a, st);
  prof_end(st);
  return e;
}

}  // namespace sr3d
