// PSF estimation (Sec. IV-B: the PSF of the real data is a fitted 3D
// Gaussian; the paper gives the fitted widths only). Given an HR reference x
// and the LR volume y, the separable sampled Gaussian H_sigma (fixed support
// of 2R+1 taps per axis), gain alpha and offset beta minimise
//   f = 1/2 ||y - alpha D H_sigma x - beta||^2.
// By eq. (8) the LR spectrum of D H_sigma x at j is (1/d) sum_a Lambda_a X_a
// over the alias group of j, with Lambda_k = l_m(k_m) l_n(k_n) l_s(k_s) the
// product of the 1D kernels' DFTs (real: the kernels are symmetric). The
// offset only moves the zero frequency, so it is fitted exactly by leaving
// j = 0 out: f = (1/(2 N_l)) sum_{j != 0} |Y_j - alpha m_j|^2 (LR Parseval),
// m_j = (1/d) sum_a Lambda_a X_a. One pass over the HR half spectrum X per
// Gauss-Newton step forms, per group, m_j, the residual r_j and the Jacobian
// row J_j = (alpha dm_j/dsigma_m, alpha dm_j/dsigma_n, alpha dm_j/dsigma_s,
// m_j), and sums Re(J^H J) (10), Re(J^H r) (4), |r|^2 and m_0 (for beta) in
// FP64.
#include "sr3d_internal.h"

namespace sr3d {

namespace {

constexpr int kPsfSums = 17;  // JtJ (10, upper triangle row-major), Jtr (4), |r|^2, m_0 (re, im)

// tab: l_m[M] | l_n[N] | l_s[S] | dl_m[M] | dl_n[N] | dl_s[S]
__global__ __launch_bounds__(kThreads) void k_psf_fit_sums(const float2 *__restrict__ X,
                                                           const float2 *__restrict__ Yh,
                                                           const float *__restrict__ tab,
                                                           float alpha, int S, int N, int M,
                                                           int dr, int dc, int ds,
                                                           double *__restrict__ part) {
  const int Mh = M / 2 + 1, Sl = S / ds, Nl = N / dc, Ml = M / dr, Mlh = Ml / 2 + 1;
  const long n = (long)Sl * Nl * Mlh;
  const float *lm = tab, *ln = tab + M, *ls = tab + M + N;
  const float *dlm = tab + M + N + S, *dln = dlm + M, *dls = dln + N;
  double acc[kPsfSums];
#pragma unroll
  for (int q = 0; q < kPsfSums; ++q) acc[q] = 0.0;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    const int jm = (int)(i % Mlh);
    const long r1 = i / Mlh;
    const int jn = (int)(r1 % Nl), js = (int)(r1 / Nl);
    // m, and the sums for its derivatives along each axis's sigma
    float2 m = make_float2(0.f, 0.f), gm = m, gn = m, gs = m;
    for (int c = 0; c < ds; ++c) {
      const int ks = js + c * Sl;
      for (int b = 0; b < dc; ++b) {
        const int kn = jn + b * Nl;
        for (int a = 0; a < dr; ++a) {
          const int km = jm + a * Ml;
          float2 x;
          if (km < Mh) {
            x = X[((long)ks * N + kn) * Mh + km];
          } else {
            x = X[((long)((S - ks) % S) * N + (N - kn) % N) * Mh + (M - km)];
            x.y = -x.y;
          }
          const float vm = lm[km], vn = ln[kn], vs = ls[ks];
          const float l = vm * vn * vs;
          const float wm = dlm[km] * vn * vs, wn = vm * dln[kn] * vs, ws = vm * vn * dls[ks];
          m.x += l * x.x; m.y += l * x.y;
          gm.x += wm * x.x; gm.y += wm * x.y;
          gn.x += wn * x.x; gn.y += wn * x.y;
          gs.x += ws * x.x; gs.y += ws * x.y;
        }
      }
    }
    const float inv_d = 1.0f / (float)(dr * dc * ds);
    const double jr[4] = {(double)(alpha * gm.x * inv_d), (double)(alpha * gn.x * inv_d),
                          (double)(alpha * gs.x * inv_d), (double)(m.x * inv_d)};
    const double ji[4] = {(double)(alpha * gm.y * inv_d), (double)(alpha * gn.y * inv_d),
                          (double)(alpha * gs.y * inv_d), (double)(m.y * inv_d)};
    if (i == 0) {  // the zero frequency: only m_0, for the offset
      acc[15] += jr[3];
      acc[16] += ji[3];
      continue;
    }
    const float2 y = Yh[i];
    const double rr = (double)y.x - (double)alpha * jr[3], ri = (double)y.y - (double)alpha * ji[3];
    // multiplicity in the full LR spectrum: 2 unless -j is stored too
    const double w = (jm == 0 || 2 * jm == Ml) ? 1.0 : 2.0;
    int q = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = u; v < 4; ++v) acc[q++] += w * (jr[u] * jr[v] + ji[u] * ji[v]);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[10 + u] += w * (jr[u] * rr + ji[u] * ri);
    acc[14] += w * (rr * rr + ri * ri);
  }
  __shared__ double sh[kThreads / 64];
#pragma unroll
  for (int q = 0; q < kPsfSums; ++q) {
    double v = acc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < kThreads / 64; ++k) t += sh[k];
      part[(long)q * gridDim.x + blockIdx.x] = t;
    }
  }
}

__global__ __launch_bounds__(1024) void k_psf_fit_reduce(const double *__restrict__ part, int nb,
                                                         double *__restrict__ out) {
  __shared__ double sh[16];
  for (int q = 0; q < kPsfSums; ++q) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 1024) v += part[(long)q * nb + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < 16; ++k) t += sh[k];
      out[q] = t;
    }
  }
}

}  // namespace

int psf_fit_blocks(long nlspec) {
  const long b = (nlspec + kThreads - 1) / kThreads;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

int psf_fit_nsums() { return kPsfSums; }

hipError_t psf_fit_sums(const float2 *X, const float2 *Yh, const float *tab, float alpha, int S,
                        int N, int M, int dr, int dc, int ds, double *part, double *out,
                        hipStream_t st) {
  const long nl = (long)(S / ds) * (N / dc) * ((M / dr) / 2 + 1);
  const int nb = psf_fit_blocks(nl);
  hipLaunchKernelGGL(k_psf_fit_sums, dim3(nb), dim3(kThreads), 0, st, X, Yh, tab, alpha, S, N, M,
                     dr, dc, ds, part);
  hipLaunchKernelGGL(k_psf_fit_reduce, dim3(1), dim3(1024), 0, st, part, nb, out);
  return hipGetLastError();
}

}  // namespace sr3d
