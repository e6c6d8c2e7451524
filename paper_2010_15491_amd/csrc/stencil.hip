// Difference / isotropic shrink / dual update (Algorithm 1 steps 5b, 5c), the
// Theta = L^T (u - d) of the next step 5a, and the residual reductions of the
// stopping rule, fused into one pass over the volume.
//
// The ADMM state (u, d) is carried as nu = L x + d_prev (3 planes): step 5b
// gives u = shrink(nu) and step 5c gives d = d_prev + (L x - u) = nu - u, so
// (u, d) are functions of nu alone. One iteration reads x and nu_old and
// writes nu_new and Theta (32 bytes per voxel); nu is double-buffered because
// neighbouring workgroups read nu_old across tile borders.
//
// A workgroup owns an 8 (n) x 64 (m) column tile and marches along s through
// a chunk of planes. Per plane it stages x with a one-voxel ring in LDS
// (forward differences), recomputes nu_new, u, d on the tile plus its lower
// n and m faces (the backward neighbours L^T needs), and keeps the s-component
// of the previous plane in registers, so the s halo costs nothing.
#include "reduce.h"

// No FMA contraction in this file: the resume path (k_theta_from_nu) must
// reproduce the fused kernel's Theta bit for bit, which requires both to round
// every product and sum the same way.
#pragma clang fp contract(off)
#include "stencil_core.h"

namespace sr3d {

constexpr int FT_M = 64, FT_N = 8, FT_COLS = FT_M * FT_N;  // tile columns (2 per thread)
constexpr int XR_M = FT_M + 2, XR_N = FT_N + 2, XR = XR_M * XR_N;  // x plane with ring
constexpr int FF_M = FT_M + 1, FF_N = FT_N + 1, FF = FF_M * FF_N;  // tile + lower faces
constexpr int NFACE = FF - FT_COLS;
constexpr int XR_PT = (XR + kThreads - 1) / kThreads;

template <bool ANISO>
__device__ __forceinline__ void point_update(const float *xc, const float *xn, int ri, float o0,
                                             float o1, float o2, float thr, PointQ &q) {
  point_update_at<ANISO>(xc, xn, ri, ri + 1, ri + XR_M, o0, o1, o2, thr, q);
}

template <typename Acc, bool STATS, bool ANISO>
__device__ __forceinline__ void stencil_body(const AdmmStencilArgs &a, const StencilPlan &pl, int b,
                                             int slot) {
  __shared__ float xs[3][XR];
  __shared__ float fw[2][FF], fd[2][FF], fu[2][FF];  // m and n components at tile + faces
  __shared__ Acc sh[6 * 4];

  const int S = a.S, N = a.N, M = a.M;
  const long NT = (long)S * N * M;
  const long plane = (long)N * M;
  const int tm = b % pl.tiles_m;
  const int tn = (b / pl.tiles_m) % pl.tiles_n;
  const int ch = b / (pl.tiles_m * pl.tiles_n);
  const int m0 = tm * FT_M, n0 = tn * FT_N;
  const int s0 = ch * pl.L;
  const int s1 = min(s0 + pl.L, S);
  const int tid = threadIdx.x;

  // Ring load items: global 2D offsets (fixed for every plane).
  long roff[XR_PT];
  int ridx[XR_PT];
#pragma unroll
  for (int k = 0; k < XR_PT; ++k) {
    const int r = tid + k * kThreads;
    ridx[k] = r;
    if (r < XR) {
      const int rn = r / XR_M, rm = r % XR_M;
      const int gn = ((n0 + rn - 1) % N + N) % N;
      const int gm = ((m0 + rm - 1) % M + M) % M;
      roff[k] = (long)gn * M + gm;
    } else {
      roff[k] = 0;
    }
  }
  // Own tile points (2) and an optional face point.
  int pl_ln[2], pl_lm[2];
  long poff[2];
  bool pval[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int c = tid + k * kThreads;
    pl_ln[k] = c / FT_M;
    pl_lm[k] = c % FT_M;
    const int gn = n0 + pl_ln[k], gm = m0 + pl_lm[k];
    pval[k] = gn < N && gm < M;
    poff[k] = (long)(gn % N) * M + (gm % M);
  }
  const bool has_face = tid < NFACE;
  int f_ln = 0, f_lm = 0;
  long foff = 0;
  if (has_face) {
    if (tid < FF_M) {
      f_ln = -1;
      f_lm = tid - 1;
    } else {
      f_ln = tid - FF_M;
      f_lm = -1;
    }
    const int gn = ((n0 + f_ln) % N + N) % N, gm = ((m0 + f_lm) % M + M) % M;
    foff = (long)gn * M + gm;
  }

  // Global loads are issued one plane ahead (x ring into registers, then LDS;
  // nu_old of the next plane into registers) so their latency overlaps the
  // arithmetic of the current plane.
  auto ring_fetch = [&](int sp, float *xr) {
    const int sg = ((sp % S) + S) % S;
    const long base = (long)sg * plane;
#pragma unroll
    for (int k = 0; k < XR_PT; ++k)
      xr[k] = (a.x && ridx[k] < XR) ? a.x[base + roff[k]] : 0.f;
  };
  auto ring_store = [&](int buf, const float *xr) {
#pragma unroll
    for (int k = 0; k < XR_PT; ++k)
      if (ridx[k] < XR) xs[buf][ridx[k]] = xr[k];
  };
  // nu_old at the 2 tile points and the face point of plane sp. The tile
  // points' state is streamed (non-temporal, as are the stores of nu_new):
  // read and written once per iteration, it would only displace the spectrum
  // and x from the last-level cache. The face points, which a neighbouring
  // tile reads too, are not.
  auto nu_fetch = [&](int sp, float (*o)[3]) {
    const long sb = (long)(((sp % S) + S) % S) * plane;
    const long offs[3] = {sb + poff[0], sb + poff[1], sb + foff};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (a.nu_in && k < 2) {
        o[k][0] = __builtin_nontemporal_load(a.nu_in + offs[k]);
        o[k][1] = __builtin_nontemporal_load(a.nu_in + offs[k] + NT);
        o[k][2] = __builtin_nontemporal_load(a.nu_in + offs[k] + 2 * NT);
      } else if (a.nu_in && has_face) {
        o[k][0] = a.nu_in[offs[k]];
        o[k][1] = a.nu_in[offs[k] + NT];
        o[k][2] = a.nu_in[offs[k] + 2 * NT];
      } else {
        o[k][0] = o[k][1] = o[k][2] = 0.f;
      }
    }
  };

  // Each thread sums its own points (at most 2 per plane over <= 32 planes)
  // in FP32; the sums across threads, workgroups and the volume are in Acc.
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float pw[2], pd[2], pu[2];  // s-components at the previous plane
  float xr[XR_PT];
  float nuc[3][3], nun[3][3];

  // Prologue: plane s0 - 1 (its s-components feed L^T at plane s0).
  {
    float xa[XR_PT], nup[3][3];
    ring_fetch(s0 - 1, xa);
    ring_fetch(s0, xr);
    nu_fetch(s0 - 1, nup);
    ring_store(0, xa);
    ring_store(1, xr);
    ring_fetch(s0 + 1, xr);
    nu_fetch(s0, nuc);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      PointQ q;
      point_update<ANISO>(xs[0], xs[1], (pl_ln[k] + 1) * XR_M + pl_lm[k] + 1, nup[k][0], nup[k][1],
                   nup[k][2], a.thr, q);
      pw[k] = q.w[2];
      pd[k] = q.d[2];
      pu[k] = q.du[2];
    }
  }

  for (int sp = s0; sp < s1; ++sp) {
    const int bc = (sp - s0 + 1) % 3, bn = (sp - s0 + 2) % 3;
    ring_store(bn, xr);  // plane sp + 1
    if (sp + 1 < s1) {
      ring_fetch(sp + 2, xr);
      nu_fetch(sp + 1, nun);
    }
    __syncthreads();
    const long sb = (long)sp * plane;
    float tw[2], td[2], tu[2];  // s-term minus the point's own sum
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      PointQ q;
      const int ri = (pl_ln[k] + 1) * XR_M + pl_lm[k] + 1;
      point_update<ANISO>(xs[bc], xs[bn], ri, nuc[k][0], nuc[k][1], nuc[k][2], a.thr, q);
      const int fi = (pl_ln[k] + 1) * FF_M + pl_lm[k] + 1;
      fw[0][fi] = q.w[0];
      fw[1][fi] = q.w[1];
      fd[0][fi] = q.d[0];
      fd[1][fi] = q.d[1];
      fu[0][fi] = q.du[0];
      fu[1][fi] = q.du[1];
      tw[k] = pw[k] - (q.w[0] + q.w[1] + q.w[2]);
      td[k] = pd[k] - (q.d[0] + q.d[1] + q.d[2]);
      tu[k] = pu[k] - (q.du[0] + q.du[1] + q.du[2]);
      pw[k] = q.w[2];
      pd[k] = q.d[2];
      pu[k] = q.du[2];
      if (pval[k]) {
        const long v = sb + poff[k];
        __builtin_nontemporal_store(q.nn[0], a.nu_out + v);
        __builtin_nontemporal_store(q.nn[1], a.nu_out + v + NT);
        __builtin_nontemporal_store(q.nn[2], a.nu_out + v + 2 * NT);
        if (STATS) {
          point_stats<ANISO>(q, acc);
        }
      }
    }
    if (has_face) {
      PointQ q;
      point_update<ANISO>(xs[bc], xs[bn], (f_ln + 1) * XR_M + f_lm + 1, nuc[2][0], nuc[2][1], nuc[2][2],
                   a.thr, q);
      const int fi = (f_ln + 1) * FF_M + f_lm + 1;
      fw[0][fi] = q.w[0];
      fw[1][fi] = q.w[1];
      fd[0][fi] = q.d[0];
      fd[1][fi] = q.d[1];
      fu[0][fi] = q.du[0];
      fu[1][fi] = q.du[1];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int fi = (pl_ln[k] + 1) * FF_M + pl_lm[k] + 1;
      // (L^T z)[i] = (z_m[i - e_m] + z_n[i - e_n]) + (z_s[i - e_s] - sum_a z_a[i])
      const float ltw = (fw[0][fi - 1] + fw[1][fi - FF_M]) + tw[k];
      const float ltd = (fd[0][fi - 1] + fd[1][fi - FF_M]) + td[k];
      const float ltu = (fu[0][fi - 1] + fu[1][fi - FF_M]) + tu[k];
      if (pval[k]) {
        a.theta[sb + poff[k]] = ltw;
        if (STATS) {
          acc[4] = fmaf(ltu, ltu, acc[4]);
          acc[5] = fmaf(ltd, ltd, acc[5]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) nuc[k][c] = nun[k][c];
  }
  if (STATS) {
    Acc acc_t[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) acc_t[q] = (Acc)acc[q];
    block_reduce_n<Acc>(acc_t, 6, sh);
    if (tid == 0) {
      Acc *p = reinterpret_cast<Acc *>(a.part);
      for (int q = 0; q < 6; ++q) p[(long)q * pl.blocks + slot] = acc_t[q];
    }
  }
}

template <typename Acc, bool STATS, bool ANISO>
__global__ __launch_bounds__(kThreads) void k_admm_stencil(AdmmStencilArgs a, StencilPlan pl) {
  if (a.done && *a.done) return;
  stencil_body<Acc, STATS, ANISO>(a, pl, xcd_tile(blockIdx.x, pl.blocks), blockIdx.x);
}

// Batch: item (volume, tile); iteration k reads nu[(k-1)&1] and writes nu[k&1].
template <typename Acc, bool ANISO>
__global__ __launch_bounds__(kThreads) void k_admm_stencil_batch(const BatchStencilDesc *__restrict__ descs,
                                                                 const int2 *__restrict__ items,
                                                                 int k) {
  const int2 it = items[blockIdx.x];
  const BatchStencilDesc d = descs[it.x];
  if (d.a.done && *d.a.done) return;
  AdmmStencilArgs a = d.a;
  // A select, not an index into the local copy (which would put it in scratch).
  float *const nu0 = d.nu[0], *const nu1 = d.nu[1];
  a.nu_in = (k & 1) ? nu0 : nu1;
  a.nu_out = (k & 1) ? nu1 : nu0;
  stencil_body<Acc, true, ANISO>(a, d.pl, it.y, it.y);
}

StencilPlan stencil_plan(int S, int N, int M) {
  StencilPlan p;
  p.tiles_m = (M + FT_M - 1) / FT_M;
  p.tiles_n = (N + FT_N - 1) / FT_N;
  const long cols = (long)p.tiles_m * p.tiles_n;
  // planes per workgroup: about 1024 workgroups, 2..32 planes (the s-halo
  // re-read is 2 planes per chunk)
  long L = (S * cols + 1023) / 1024;
  if (L < 2) L = 2;
  if (L > 32) L = 32;
  if (L > S) L = S;
  p.L = (int)L;
  p.chunks = (S + p.L - 1) / p.L;
  p.blocks = (int)(cols * p.chunks);
  return p;
}

template <bool ANISO>
static void launch_stencil_batch(const BatchStencilDesc *descs, const int2 *items, int nitems,
                                 int k, bool fp64, hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL((k_admm_stencil_batch<double, ANISO>), dim3(nitems), dim3(kThreads), 0, st,
                       descs, items, k);
  else
    hipLaunchKernelGGL((k_admm_stencil_batch<float, ANISO>), dim3(nitems), dim3(kThreads), 0, st,
                       descs, items, k);
}

hipError_t admm_stencil_batch(const BatchStencilDesc *descs, const int2 *items, int nitems, int k,
                              bool fp64, bool aniso, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  if (aniso) launch_stencil_batch<true>(descs, items, nitems, k, fp64, st);
  else launch_stencil_batch<false>(descs, items, nitems, k, fp64, st);
  return hipGetLastError();
}

template <bool ANISO>
static void launch_stencil(const AdmmStencilArgs &a, const StencilPlan &pl, bool stats, bool fp64,
                           hipStream_t st) {
  dim3 g(pl.blocks), b(kThreads);
  if (stats) {
    if (fp64) hipLaunchKernelGGL((k_admm_stencil<double, true, ANISO>), g, b, 0, st, a, pl);
    else hipLaunchKernelGGL((k_admm_stencil<float, true, ANISO>), g, b, 0, st, a, pl);
  } else {
    hipLaunchKernelGGL((k_admm_stencil<float, false, ANISO>), g, b, 0, st, a, pl);
  }
}

hipError_t admm_stencil(const AdmmStencilArgs &a, bool stats, bool fp64, hipStream_t st) {
  const StencilPlan pl = stencil_plan(a.S, a.N, a.M);
  prof_begin(kStStencil, st);
  if (a.aniso) launch_stencil<true>(a, pl, stats, fp64, st);
  else launch_stencil<false>(a, pl, stats, fp64, st);
  hipError_t e = hipGetLastError();
  prof_end(st);
  return e;
}

// Theta = L^T (u - d) of a given state nu (resuming from a checkpoint).
template <bool ANISO>
__global__ __launch_bounds__(kThreads) void k_theta_from_nu(const float *__restrict__ nu,
                                                            float *__restrict__ theta, int S, int N,
                                                            int M, float thr) {
  const long NT = (long)S * N * M;
  const long v = (long)blockIdx.x * kThreads + threadIdx.x;
  if (v >= NT) return;
  const int im = (int)(v % M);
  const long r = v / M;
  const int in = (int)(r % N), is = (int)(r / N);
  const long plane = (long)N * M;
  const long nb[3] = {v + ((im == 0) ? (long)(M - 1) : -1L),
                      v + ((in == 0) ? (long)(N - 1) * M : -(long)M),
                      v + ((is == 0) ? (long)(S - 1) * plane : -plane)};
  // Same operation order as k_admm_stencil, so a resumed solve continues the
  // iteration bit for bit.
  float u[3], w[3], nb_w[3];
  const float p[3] = {nu[v], nu[v + NT], nu[v + 2 * NT]};
  shrink_tv<ANISO>(p[0], p[1], p[2], thr, u[0], u[1], u[2]);
  for (int c = 0; c < 3; ++c) {
    const float d = p[c] - u[c];
    w[c] = u[c] - d;
  }
  const float sw = w[0] + w[1] + w[2];
  for (int c = 0; c < 3; ++c) {
    float q[3];
    const float s[3] = {nu[nb[c]], nu[nb[c] + NT], nu[nb[c] + 2 * NT]};
    shrink_tv<ANISO>(s[0], s[1], s[2], thr, q[0], q[1], q[2]);
    const float d = s[c] - q[c];
    nb_w[c] = q[c] - d;
  }
  // (L^T w)[i] = (w_m[i - e_m] + w_n[i - e_n]) + (w_s[i - e_s] - sum_a w_a[i])
  const float t = (nb_w[0] + nb_w[1]) + (nb_w[2] - sw);
  theta[v] = t;
}

hipError_t theta_from_nu(const float *nu, float *theta, int S, int N, int M, float thr,
                         bool aniso, hipStream_t st) {
  const long NT = (long)S * N * M;
  const dim3 g((unsigned)((NT + kThreads - 1) / kThreads));
  if (aniso)
    hipLaunchKernelGGL(k_theta_from_nu<true>, g, dim3(kThreads), 0, st, nu, theta, S, N, M, thr);
  else
    hipLaunchKernelGGL(k_theta_from_nu<false>, g, dim3(kThreads), 0, st, nu, theta, S, N, M, thr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final reduction and stopping rule (one workgroup).
// ---------------------------------------------------------------------------

template <typename Acc>
__global__ __launch_bounds__(1024) void k_reduce_test(Ctrl *c, const Acc *ps, int nbs,
                                                      const Acc *pf, int nbf) {
  if (c->done) return;
  reduce_body<Acc, 1024>(c, ps, nbs, pf, nbf);
}

// Batch: one workgroup per volume. When a volume stops (converged, capped or
// failed, here or earlier in the fold), the count of active volumes drops by
// one, exactly once per volume.
template <typename Acc>
__global__ __launch_bounds__(1024) void k_reduce_test_batch(const ReduceDesc *__restrict__ descs,
                                                            int *active) {
  const ReduceDesc d = descs[blockIdx.x];
  Ctrl *c = d.ctrl;
  if (!c->done) {
    reduce_body<Acc, 1024>(c, (const Acc *)d.ps, d.nbs, (const Acc *)d.pf, d.nbf);
    __syncthreads();
  }
  if (threadIdx.x == 0 && c->done && !c->counted) {
    c->counted = 1;
    atomicSub(active, 1);
  }
}

hipError_t reduce_and_test_batch(const ReduceDesc *descs, int nvol, int *active, bool fp64,
                                 hipStream_t st) {
  if (fp64)
    hipLaunchKernelGGL(k_reduce_test_batch<double>, dim3(nvol), dim3(1024), 0, st, descs, active);
  else
    hipLaunchKernelGGL(k_reduce_test_batch<float>, dim3(nvol), dim3(1024), 0, st, descs, active);
  return hipGetLastError();
}

hipError_t reduce_and_test(Ctrl *ctrl, const void *partS, int nbS, const void *partF, int nbF,
                           bool fp64, hipStream_t st) {
  prof_begin(kStReduce, st);
  if (fp64)
    hipLaunchKernelGGL(k_reduce_test<double>, dim3(1), dim3(1024), 0, st, ctrl,
                       (const double *)partS, nbS, (const double *)partF, nbF);
  else
    hipLaunchKernelGGL(k_reduce_test<float>, dim3(1), dim3(1024), 0, st, ctrl,
                       (const float *)partS, nbS, (const float *)partF, nbF);
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

__global__ void k_ctrl_init(Ctrl *c, int max_iter, float tol, float tol_dual, float mu, float lam,
                            double inv_nl) {
  if (threadIdx.x != 0) return;
  c->done = 0;
  c->iter = 0;
  c->converged = 0;
  c->status = 0;
  c->max_iter = max_iter;
  c->counted = 0;
  c->tol = tol;
  c->mu = mu;
  c->lam = lam;
  c->tol_dual = tol_dual > 0.f ? tol_dual : tol;
  c->primal_rel = INFINITY;
  c->dual_rel = INFINITY;
  c->objective = 0.0;
  c->inv_nl = inv_nl;
}

hipError_t ctrl_init(Ctrl *c, int max_iter, float tol, float tol_dual, float mu, float lam,
                     double inv_nl, hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, c, max_iter, tol, tol_dual, mu, lam,
                     inv_nl);
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

__global__ void k_add_to(float *y, const float *x, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

hipError_t add_to(float *y, const float *x, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_add_to, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, x, (long)n);
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
