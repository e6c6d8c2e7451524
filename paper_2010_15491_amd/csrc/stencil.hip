// Difference / isotropic shrink / dual update (Algorithm 1 steps 5b, 5c) and
// the Theta = L^T (u - d) of the next step 5a, plus the residual reductions of
// the stopping rule.
//
// The ADMM state (u, d) is carried as nu = L x + d_prev (3 planes): step 5b
// gives u = shrink(nu) and step 5c gives d = d_prev + (L x - u) = nu - u, so
// (u, d) are functions of nu alone. This halves the state traffic.
//
// stencil_a (per voxel i): L x with periodic forward differences,
//   nu' = L x + d(nu), u' = shrink(nu'), accumulates |Lx-u'|^2 (= |d'-d|^2),
//   |Lx|^2, |u'|^2 and the TV term |(Lx)_i|.
// stencil_b (per voxel i): u', d' at i and at i - e_a (a = m, n, s),
//   Theta = L^T u' - L^T d', accumulates |L^T u' - L^T u|^2 and |L^T d'|^2,
//   and stores L^T u' for the next dual residual.
// Each workgroup covers kStencilVox consecutive voxels, taken in an XCD-aware
// order so the planes a workgroup touches stay in one XCD's L2.
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
  if (lane == 0)
    for (int q = 0; q < n; ++q) sh[q * 4 + wid] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int q = 0; q < n; ++q) v[q] = sh[q * 4 + 0] + sh[q * 4 + 1] + sh[q * 4 + 2] + sh[q * 4 + 3];
}

// Workgroup b of nb is dispatched to XCD b % 8; give every XCD a contiguous
// range of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, l = b >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

__device__ __forceinline__ void shrink3(float a0, float a1, float a2, float thr, float &u0,
                                        float &u1, float &u2) {
  const float n2 = a0 * a0 + a1 * a1 + a2 * a2;
  float s = 0.f;
  if (n2 > 0.f) {
    const float n = sqrtf(n2);
    s = fmaxf(n - thr, 0.f) / n;
  }
  u0 = a0 * s;
  u1 = a1 * s;
  u2 = a2 * s;
}

template <typename Acc, int MODE>
__global__ __launch_bounds__(kThreads) void k_stencil_a(StencilArgs a, FastDiv divM, FastDiv divN,
                                                        int nb) {
  if (a.done && *a.done) return;
  __shared__ Acc sh[4 * 4];
  const long NT = (long)a.S * a.N * a.M;
  const long plane = (long)a.N * a.M;
  const int tile = xcd_tile(blockIdx.x, nb);
  Acc acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < kStencilVpt; ++k) {
    const long v = (long)tile * kStencilVox + k * kThreads + threadIdx.x;
    if (v >= NT) break;
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
    if (MODE != 2) {
      const uint32_t r1 = divM.div((uint32_t)v);
      const int im = (int)(v - (long)r1 * a.M);
      const uint32_t is = divN.div(r1);
      const int in = (int)(r1 - is * (uint32_t)a.N);
      const long om = (im + 1 == a.M) ? -(long)(a.M - 1) : 1;
      const long on = (in + 1 == a.N) ? -(long)(a.N - 1) * a.M : (long)a.M;
      const long os = ((int)is + 1 == a.S) ? -(long)(a.S - 1) * plane : plane;
      const float xi = a.x[v];
      const float l0 = a.x[v + om] - xi, l1 = a.x[v + on] - xi, l2 = a.x[v + os] - xi;
      float d0 = 0.f, d1 = 0.f, d2 = 0.f;
      if (MODE == 0) {
        const float p0 = a.nu[v], p1 = a.nu[v + NT], p2 = a.nu[v + 2 * NT];
        float u0, u1, u2;
        shrink3(p0, p1, p2, a.thr, u0, u1, u2);
        d0 = p0 - u0;
        d1 = p1 - u1;
        d2 = p2 - u2;
      }
      n0 = l0 + d0;
      n1 = l1 + d1;
      n2 = l2 + d2;
      if (MODE == 0) {
        float u0, u1, u2;
        shrink3(n0, n1, n2, a.thr, u0, u1, u2);
        const float r0 = l0 - u0, r1_ = l1 - u1, r2 = l2 - u2;
        const Acc lx2 = (Acc)l0 * l0 + (Acc)l1 * l1 + (Acc)l2 * l2;
        acc[0] += (Acc)r0 * r0 + (Acc)r1_ * r1_ + (Acc)r2 * r2;
        acc[1] += lx2;
        acc[2] += (Acc)u0 * u0 + (Acc)u1 * u1 + (Acc)u2 * u2;
        acc[3] += sqrt(lx2);
      }
    }
    a.nu[v] = n0;
    a.nu[v + NT] = n1;
    a.nu[v + 2 * NT] = n2;
  }
  if (MODE == 0) {
    block_reduce_n<Acc>(acc, 4, sh);
    if (threadIdx.x == 0) {
      Acc *p = reinterpret_cast<Acc *>(a.partA);
      for (int q = 0; q < 4; ++q) p[(long)q * nb + blockIdx.x] = acc[q];
    }
  }
}

template <typename Acc, int INIT>
__global__ __launch_bounds__(kThreads) void k_stencil_b(StencilArgs a, FastDiv divM, FastDiv divN,
                                                        int nb) {
  if (a.done && *a.done) return;
  __shared__ Acc sh[2 * 4];
  const long NT = (long)a.S * a.N * a.M;
  const long plane = (long)a.N * a.M;
  const int tile = xcd_tile(blockIdx.x, nb);
  Acc acc[2] = {0, 0};
  for (int k = 0; k < kStencilVpt; ++k) {
    const long v = (long)tile * kStencilVox + k * kThreads + threadIdx.x;
    if (v >= NT) break;
    const uint32_t r1 = divM.div((uint32_t)v);
    const int im = (int)(v - (long)r1 * a.M);
    const uint32_t is = divN.div(r1);
    const int in = (int)(r1 - is * (uint32_t)a.N);
    const long om = (im == 0) ? (long)(a.M - 1) : -1;
    const long on = (in == 0) ? (long)(a.N - 1) * a.M : -(long)a.M;
    const long os = (is == 0) ? (long)(a.S - 1) * plane : -plane;
    float u0, u1, u2;
    const float p0 = a.nu[v], p1 = a.nu[v + NT], p2 = a.nu[v + 2 * NT];
    shrink3(p0, p1, p2, a.thr, u0, u1, u2);
    float ltu = -(u0 + u1 + u2);
    float ltd = -((p0 - u0) + (p1 - u1) + (p2 - u2));
    {
      const long w = v + om;
      float q0, q1, q2;
      const float s0 = a.nu[w], s1 = a.nu[w + NT], s2 = a.nu[w + 2 * NT];
      shrink3(s0, s1, s2, a.thr, q0, q1, q2);
      ltu += q0;
      ltd += s0 - q0;
    }
    {
      const long w = v + on;
      float q0, q1, q2;
      const float s0 = a.nu[w], s1 = a.nu[w + NT], s2 = a.nu[w + 2 * NT];
      shrink3(s0, s1, s2, a.thr, q0, q1, q2);
      ltu += q1;
      ltd += s1 - q1;
    }
    {
      const long w = v + os;
      float q0, q1, q2;
      const float s0 = a.nu[w], s1 = a.nu[w + NT], s2 = a.nu[w + 2 * NT];
      shrink3(s0, s1, s2, a.thr, q0, q1, q2);
      ltu += q2;
      ltd += s2 - q2;
    }
    if (!INIT) {
      const float old = a.ltu[v];
      const float du = ltu - old;
      acc[0] += (Acc)du * du;
      acc[1] += (Acc)ltd * ltd;
    }
    a.ltu[v] = ltu;
    a.theta[v] = ltu - ltd;
  }
  if (!INIT) {
    block_reduce_n<Acc>(acc, 2, sh);
    if (threadIdx.x == 0) {
      Acc *p = reinterpret_cast<Acc *>(a.partB);
      for (int q = 0; q < 2; ++q) p[(long)q * nb + blockIdx.x] = acc[q];
    }
  }
}

int stencil_blocks(int S, int N, int M) {
  const long NT = (long)S * N * M;
  return (int)((NT + kStencilVox - 1) / kStencilVox);
}

hipError_t stencil_a(const StencilArgs &a, int mode, bool fp64, hipStream_t st) {
  const int nb = stencil_blocks(a.S, a.N, a.M);
  FastDiv dm((uint32_t)a.M), dn((uint32_t)a.N);
  dim3 g(nb), b(kThreads);
  prof_begin(kStStencilA, st);
#define SR3D_LA(ACC, MD) hipLaunchKernelGGL((k_stencil_a<ACC, MD>), g, b, 0, st, a, dm, dn, nb)
  if (fp64) {
    if (mode == 0) SR3D_LA(double, 0);
    else if (mode == 1) SR3D_LA(double, 1);
    else SR3D_LA(double, 2);
  } else {
    if (mode == 0) SR3D_LA(float, 0);
    else if (mode == 1) SR3D_LA(float, 1);
    else SR3D_LA(float, 2);
  }
#undef SR3D_LA
  hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

hipError_t stencil_b(const StencilArgs &a, int init, bool fp64, hipStream_t st) {
  const int nb = stencil_blocks(a.S, a.N, a.M);
  FastDiv dm((uint32_t)a.M), dn((uint32_t)a.N);
  dim3 g(nb), b(kThreads);
  prof_begin(kStStencilB, st);
#define SR3D_LB(ACC, IN) hipLaunchKernelGGL((k_stencil_b<ACC, IN>), g, b, 0, st, a, dm, dn, nb)
  if (fp64) {
    if (init) SR3D_LB(double, 1);
    else SR3D_LB(double, 0);
  } else {
    if (init) SR3D_LB(float, 1);
    else SR3D_LB(float, 0);
  }
#undef SR3D_LB
  hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

// ---------------------------------------------------------------------------
// Final reduction and stopping rule (one workgroup).
// ---------------------------------------------------------------------------

template <typename Acc>
__device__ Acc sum_range(const Acc *p, int n, Acc *sh) {
  Acc s = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = s;
  __syncthreads();
  Acc r = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

template <typename Acc>
__global__ __launch_bounds__(1024) void k_reduce_test(Ctrl *c, const Acc *pa, int nba, const Acc *pb,
                                                      int nbb, const Acc *pf, int nbf) {
  if (c->done) return;
  __shared__ Acc sh[16];
  Acc q[7];
  for (int k = 0; k < 4; ++k) q[k] = sum_range<Acc>(pa + (long)k * nba, nba, sh);
  for (int k = 0; k < 2; ++k) q[4 + k] = sum_range<Acc>(pb + (long)k * nbb, nbb, sh);
  q[6] = pf ? sum_range<Acc>(pf, nbf, sh) : (Acc)0;
  if (threadIdx.x != 0) return;
  bool finite = true;
  for (int k = 0; k < 7; ++k) finite = finite && isfinite(q[k]);
  const Acc mu = (Acc)c->mu, tol = (Acc)c->tol;
  const Acc r = sqrt(q[0]);
  const Acc pden = fmax(sqrt(q[1]), sqrt(q[2]));
  const Acc s = mu * sqrt(q[4]);
  const Acc dden = mu * sqrt(q[5]);
  const Acc inf = (Acc)INFINITY;
  const Acc prel = pden > 0 ? r / pden : inf;
  const Acc drel = dden > 0 ? s / dden : inf;
  c->iter += 1;
  c->primal_rel = (double)prel;
  c->dual_rel = (double)drel;
  c->objective = (double)((Acc)0.5 * q[6] * (Acc)c->inv_nl + (Acc)c->lam * q[3]);
  if (!finite) {
    c->status = SR3D_ERR_NONFINITE;
    c->done = 1;
    return;
  }
  if (tol > 0 && prel <= tol && drel <= tol) {
    c->converged = 1;
    c->done = 1;
  }
  if (c->iter >= c->max_iter) c->done = 1;
}

hipError_t reduce_and_test(Ctrl *ctrl, const void *partA, int nbA, const void *partB, int nbB,
                           const void *partF, int nbF, bool fp64, hipStream_t st) {
  prof_begin(kStReduce, st);
  if (fp64)
    hipLaunchKernelGGL(k_reduce_test<double>, dim3(1), dim3(1024), 0, st, ctrl,
                       (const double *)partA, nbA, (const double *)partB, nbB,
                       (const double *)partF, nbF);
  else
    hipLaunchKernelGGL(k_reduce_test<float>, dim3(1), dim3(1024), 0, st, ctrl,
                       (const float *)partA, nbA, (const float *)partB, nbB,
                       (const float *)partF, nbF);
  hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// out[i] = psf[(i + K/2) mod dims] if that index lies inside the PSF, else 0:
// the PSF zero-padded to the HR grid, centre tap moved to the origin (eq. (2)).
__global__ void k_pad_psf(const float *__restrict__ psf, int Ks, int Kn, int Km,
                          float *__restrict__ out, int S, int N, int M) {
  const long NT = (long)S * N * M;
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= NT) return;
  const int im = (int)(v % M);
  const long r = v / M;
  const int in = (int)(r % N), is = (int)(r / N);
  const int pm = (im + Km / 2) % M, pn = (in + Kn / 2) % N, ps = (is + Ks / 2) % S;
  float val = 0.f;
  if (pm < Km && pn < Kn && ps < Ks) val = psf[((long)ps * Kn + pn) * Km + pm];
  out[v] = val;
}

hipError_t pad_psf(const float *psf, int Ks, int Kn, int Km, float *out, int S, int N, int M,
                   hipStream_t st) {
  const long NT = (long)S * N * M;
  hipLaunchKernelGGL(k_pad_psf, dim3((unsigned)((NT + 255) / 256)), dim3(256), 0, st, psf, Ks, Kn,
                     Km, out, S, N, M);
  return hipGetLastError();
}

// |e^{2 pi i k/n} - 1|^2 = 4 sin^2(pi k / n) per axis, computed in FP64.
__global__ void k_diff_tables(float *g, int S, int N, int M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int tot = M + N + S;
  if (i >= tot) return;
  int k, n;
  if (i < M) { k = i; n = M; }
  else if (i < M + N) { k = i - M; n = N; }
  else { k = i - M - N; n = S; }
  const double sv = sin(M_PI * (double)k / (double)n);
  g[i] = (float)(4.0 * sv * sv);
}

hipError_t diff_tables(float *g, int S, int N, int M, hipStream_t st) {
  const int tot = M + N + S;
  hipLaunchKernelGGL(k_diff_tables, dim3((tot + 255) / 256), dim3(256), 0, st, g, S, N, M);
  return hipGetLastError();
}

__global__ void k_ctrl_init(Ctrl *c, int max_iter, float tol, float mu, float lam, double inv_nl) {
  if (threadIdx.x != 0) return;
  c->done = 0;
  c->iter = 0;
  c->converged = 0;
  c->status = 0;
  c->max_iter = max_iter;
  c->pad0 = 0;
  c->tol = tol;
  c->mu = mu;
  c->lam = lam;
  c->pad1 = 0.f;
  c->primal_rel = INFINITY;
  c->dual_rel = INFINITY;
  c->objective = 0.0;
  c->inv_nl = inv_nl;
}

hipError_t ctrl_init(Ctrl *c, int max_iter, float tol, float mu, float lam, double inv_nl,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, c, max_iter, tol, mu, lam, inv_nl);
  return hipGetLastError();
}

__global__ void k_fill_zero(float *p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

hipError_t fill_zero(float *p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, (long)n);
  return hipGetLastError();
}

__global__ void k_spectrum_mul(float2 *W, const float2 *L, long n, float scale) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 a = W[i], b = L[i];
  W[i] = make_float2((a.x * b.x - a.y * b.y) * scale, (a.x * b.y + a.y * b.x) * scale);
}

hipError_t spectrum_mul(float2 *W, const float2 *Lam, size_t n, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_spectrum_mul, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, Lam,
                     (long)n, scale);
  return hipGetLastError();
}

__global__ void k_decimate(const float *x, float *y, int S, int N, int M, int dr, int dc, int ds) {
  const int Ml = M / dr, Nl = N / dc, Sl = S / ds;
  const long NL = (long)Sl * Nl * Ml;
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= NL) return;
  const int jm = (int)(v % Ml);
  const long r = v / Ml;
  const int jn = (int)(r % Nl), js = (int)(r / Nl);
  y[v] = x[((long)js * ds * N + (long)jn * dc) * M + (long)jm * dr];
}

hipError_t decimate(const float *x, float *y, int S, int N, int M, int dr, int dc, int ds,
                    hipStream_t st) {
  const long NL = (long)(S / ds) * (N / dc) * (M / dr);
  hipLaunchKernelGGL(k_decimate, dim3((unsigned)((NL + 255) / 256)), dim3(256), 0, st, x, y, S, N,
                     M, dr, dc, ds);
  return hipGetLastError();
}

}  // namespace sr3d
