// l1 data term (non-Gaussian noise, which the paper's conclusion names as
// future work): min_x ||D H x - y||_1 + lam TV(x) by ADMM with a second split
// v = D H x - y next to u = L x. The x-step is Algorithm 1 step 5a with
// y -> y' = y + v - e and mu -> mu / mu_data, so the x-update, the FFTs and
// the TV stencil are the existing ones; this file holds the LR-grid pieces:
//   - the weights W_j = sum over the alias group of j of |Lambda_k|^2, which
//     turn an LR spectrum into the norm of its image under H^T D^T:
//     ||H^T D^T z||^2 = (1/N_h) sum_j W_j |(F z)_j|^2 (Parseval, with
//     F(D^T z)_k = (F z)_{k mod LR} for offset-0 decimation);
//   - the v/e update (steps 5b'/5c'): v' = soft(DHx - y + e, 1/mu_data),
//     e' = e + DHx - y - v', and y' for the next x-step;
//   - the weighted spectral norms of the data split's dual residual;
//   - the stopping test over both splits.
#include "reduce.h"
#include "stencil_core.h"

namespace sr3d {

namespace {

template <typename T>
__device__ __forceinline__ T wg_sum(T v, T *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// One thread per stored LR half-spectrum entry j = (js, jn, jm), jm <= Ml/2.
// W_j sums |Lambda_k|^2 over the members k = (js + c Sl, jn + b Nl, jm + a Ml)
// (read at -k where k_m > M/2: the same modulus for a real PSF). The entry's
// multiplicity in the full LR spectrum (2 where -j is not stored) is folded in.
__global__ void k_l1_weights(const float2 *__restrict__ lam, float *__restrict__ w, int S, int N,
                             int M, int Sl, int Nl, int Ml, int dr, int dc, int ds) {
  const int Mh = M / 2 + 1, Mlh = Ml / 2 + 1;
  const long n = (long)Sl * Nl * Mlh;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int jm = (int)(i % Mlh);
  const long r = i / Mlh;
  const int jn = (int)(r % Nl), js = (int)(r / Nl);
  double acc = 0.0;
  for (int c = 0; c < ds; ++c)
    for (int b = 0; b < dc; ++b)
      for (int a = 0; a < dr; ++a) {
        const int ks = js + c * Sl, kn = jn + b * Nl, km = jm + a * Ml;
        long id;
        if (km < Mh) id = ((long)ks * N + kn) * Mh + km;
        else id = ((long)((S - ks) % S) * N + (N - kn) % N) * Mh + (M - km);
        const float2 l = lam[id];
        acc += (double)l.x * l.x + (double)l.y * l.y;
      }
  const bool self = jm == 0 || 2 * jm == Ml;
  w[i] = (float)(self ? acc : 2.0 * acc);
}

// Steps 5b'/5c' on the LR grid. t = D H x; with `init` the duals are zero
// (the initialisation applies the steps to x0). Writes v', e', y' = y + v' - e'
// and dv = v' - v; partial sums per workgroup (5 arrays of nb):
//   |t - y - v'|^2, |t|^2, |v'|^2, |y|^2, sum |t - y|.
template <typename Acc>
__global__ __launch_bounds__(kThreads) void k_l1_update(const float *__restrict__ t,
                                                        const float *__restrict__ y,
                                                        float *__restrict__ v, float *__restrict__ e,
                                                        float *__restrict__ yp,
                                                        float *__restrict__ dv, long n, float thr,
                                                        int init, Acc *__restrict__ part,
                                                        const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ Acc sh[kThreads / 64];
  float q[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    const float ti = t ? t[i] : 0.f;
    const float yi = y[i];
    const float vo = init ? 0.f : v[i];
    const float eo = init ? 0.f : e[i];
    const float r = ti - yi;
    const float a = r + eo;
    const float vn = shrink1(a, thr);
    const float en = a - vn;
    v[i] = vn;
    e[i] = en;
    yp[i] = (yi + vn) - en;
    if (dv) dv[i] = vn - vo;
    const float pr = r - vn;
    q[0] += pr * pr;
    q[1] += ti * ti;
    q[2] += vn * vn;
    q[3] += yi * yi;
    q[4] += fabsf(r);
  }
  if (!part) return;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const Acc s = wg_sum<Acc>((Acc)q[k], sh);
    if (threadIdx.x == 0) part[(long)k * gridDim.x + blockIdx.x] = s;
  }
}

// sum_j W_j |A_j|^2 and sum_j W_j |B_j|^2 over the LR half spectra A = F dv,
// B = F e' (partials: 2 arrays of nb).
template <typename Acc>
__global__ __launch_bounds__(kThreads) void k_l1_wnorm(const float2 *__restrict__ A,
                                                       const float2 *__restrict__ B,
                                                       const float *__restrict__ w, long n,
                                                       Acc *__restrict__ part,
                                                       const int *__restrict__ done) {
  if (done && *done) return;
  __shared__ Acc sh[kThreads / 64];
  Acc qa = 0, qb = 0;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    const float2 a = A[i], b = B[i];
    const float wi = w[i];
    qa += (Acc)(wi * (a.x * a.x + a.y * a.y));
    qb += (Acc)(wi * (b.x * b.x + b.y * b.y));
  }
  qa = wg_sum<Acc>(qa, sh);
  qb = wg_sum<Acc>(qb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = qa;
    part[gridDim.x + blockIdx.x] = qb;
  }
}

// The 13 sums of the partial arrays (part k of an array at base + k n, n
// entries) in one pass by the one workgroup of kRedThreads: grid-stride
// loops, wavefront butterflies, then the wavefronts' totals in order.
constexpr int kRedThreads = 256;

template <typename Acc>
__device__ __forceinline__ void sum_all_parts(const Acc *ps, int nbs, const Acc *pl, int nbl,
                                              const Acc *pw, int nbw, Acc (&r)[13],
                                              Acc (*sh)[13]) {
  Acc v[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) v[k] = 0;
  for (int i = threadIdx.x; i < nbs; i += kRedThreads)
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] += ps[(long)k * nbs + i];
  for (int i = threadIdx.x; i < nbl; i += kRedThreads)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[6 + k] += pl[(long)k * nbl + i];
  for (int i = threadIdx.x; i < nbw; i += kRedThreads)
#pragma unroll
    for (int k = 0; k < 2; ++k) v[11 + k] += pw[(long)k * nbw + i];
#pragma unroll
  for (int k = 0; k < 13; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 13; ++k) sh[wid][k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 13; ++k) {
    Acc t = 0;
#pragma unroll
    for (int i = 0; i < kRedThreads / 64; ++i) t += sh[i][k];
    r[k] = t;
  }
}

// The stopping test over both splits (one workgroup). TV
// split from the stencil sums (as in the plain solve), data split:
//   primal = |DHx - y - v'| / max(|DHx|, |v'|, |y|),
//   dual   = |H^T D^T (v' - v)| / |H^T D^T e'|  (mu_data cancels),
// the reported primal and dual being the larger of the two splits'; the
// objective is sum |DHx - y| + lam TV(x).
template <typename Acc>
__global__ __launch_bounds__(kRedThreads) void k_l1_reduce_test(Ctrl *c, const Acc *ps, int nbs,
                                                         const Acc *pl, int nbl, const Acc *pw,
                                                         int nbw) {
  if (c->done) return;
  __shared__ Acc sh[kRedThreads / 64][13];
  Acc r[13];
  sum_all_parts<Acc>(ps, nbs, pl, nbl, pw, nbw, r, sh);
  if (threadIdx.x != 0) return;
  Acc q[6], l[5], w[2];
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 13; ++k) finite = finite && isfinite(r[k]);
#pragma unroll
  for (int k = 0; k < 6; ++k) q[k] = r[k];
#pragma unroll
  for (int k = 0; k < 5; ++k) l[k] = r[6 + k];
#pragma unroll
  for (int k = 0; k < 2; ++k) w[k] = r[11 + k];
  const Acc inf = (Acc)INFINITY;
  const Acc pden_tv = fmax(sqrt(q[1]), sqrt(q[2]));
  const Acc p_tv = pden_tv > 0 ? sqrt(q[0]) / pden_tv : inf;
  const Acc d_tv = q[5] > 0 ? sqrt(q[4]) / sqrt(q[5]) : inf;
  const Acc pden_da = fmax(fmax(sqrt(l[1]), sqrt(l[2])), sqrt(l[3]));
  const Acc p_da = pden_da > 0 ? sqrt(l[0]) / pden_da : inf;
  const Acc d_da = w[1] > 0 ? sqrt(w[0]) / sqrt(w[1]) : inf;
  const Acc prel = fmax(p_tv, p_da), drel = fmax(d_tv, d_da);
  c->iter += 1;
  c->primal_rel = (double)prel;
  c->dual_rel = (double)drel;
  c->objective = (double)(l[4] + (Acc)c->lam * q[3]);
  if (!finite) {
    c->status = SR3D_ERR_NONFINITE;
    c->done = 1;
    return;
  }
  const Acc tol = (Acc)c->tol, tol_d = (Acc)c->tol_dual;
  if (tol > 0 && prel <= tol && drel <= tol_d) {
    c->converged = 1;
    c->done = 1;
  }
  if (c->iter >= c->max_iter) c->done = 1;
}

}  // namespace

int l1_blocks(long n) {
  const long b = (n + kThreads - 1) / kThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t l1_weights(const float2 *lam, float *w, int S, int N, int M, int dr, int dc, int ds,
                      hipStream_t st) {
  const int Sl = S / ds, Nl = N / dc, Ml = M / dr;
  const long n = (long)Sl * Nl * (Ml / 2 + 1);
  hipLaunchKernelGGL(k_l1_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lam, w, S,
                     N, M, Sl, Nl, Ml, dr, dc, ds);
  return hipGetLastError();
}

hipError_t l1_update(const float *t, const float *y, float *v, float *e, float *yp, float *dv,
                     long n, float thr, bool init, void *part, bool fp64, const int *done,
                     hipStream_t st) {
  const int nb = l1_blocks(n);
  if (fp64)
    hipLaunchKernelGGL(k_l1_update<double>, dim3(nb), dim3(kThreads), 0, st, t, y, v, e, yp, dv, n,
                       thr, init ? 1 : 0, (double *)part, done);
  else
    hipLaunchKernelGGL(k_l1_update<float>, dim3(nb), dim3(kThreads), 0, st, t, y, v, e, yp, dv, n,
                       thr, init ? 1 : 0, (float *)part, done);
  return hipGetLastError();
}

hipError_t l1_wnorm(const float2 *A, const float2 *B, const float *w, long n, void *part, bool fp64,
                    const int *done, hipStream_t st) {
  const int nb = l1_blocks(n);
  if (fp64)
    hipLaunchKernelGGL(k_l1_wnorm<double>, dim3(nb), dim3(kThreads), 0, st, A, B, w, n,
                       (double *)part, done);
  else
    hipLaunchKernelGGL(k_l1_wnorm<float>, dim3(nb), dim3(kThreads), 0, st, A, B, w, n,
                       (float *)part, done);
  return hipGetLastError();
}

hipError_t l1_reduce_test(Ctrl *c, const void *ps, int nbs, const void *pl, int nbl, const void *pw,
                          int nbw, bool fp64, hipStream_t st) {
  prof_begin(kStReduce, st);
  if (fp64)
    hipLaunchKernelGGL(k_l1_reduce_test<double>, dim3(1), dim3(kRedThreads), 0, st, c, (const double *)ps,
                       nbs, (const double *)pl, nbl, (const double *)pw, nbw);
  else
    hipLaunchKernelGGL(k_l1_reduce_test<float>, dim3(1), dim3(kRedThreads), 0, st, c, (const float *)ps,
                       nbs, (const float *)pl, nbl, (const float *)pw, nbw);
  const hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

}  // namespace sr3d
