// Final reduction of the residual partial sums and the stopping rule
// (Algorithm 1, after step 5): shared by the reduction kernels and by the
// extra workgroup that runs it inside the next iteration's first launch.
#pragma once

#include "sr3d_internal.h"

namespace sr3d {

// Sums of the 6 stencil partial arrays and the fold partials, all loads of a
// thread issued before any shuffle.
template <typename Acc, int NT>
__device__ __forceinline__ void reduce_body(Ctrl *c, const Acc *ps, int nbs, const Acc *pf,
                                            int nbf) {
  __shared__ Acc sh[7][NT / 64];
  Acc q[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < nbs; i += NT) {
#pragma unroll
    for (int k = 0; k < 6; ++k) q[k] += ps[(long)k * nbs + i];
  }
  if (pf)
    for (int i = threadIdx.x; i < nbf; i += NT) q[6] += pf[i];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) q[k] += __shfl_xor(q[k], off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 7; ++k) sh[k][wid] = q[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < 7; ++k) {
    Acc t = 0;
    for (int w = 0; w < NT / 64; ++w) t += sh[k][w];
    q[k] = t;
  }
  bool finite = true;
  for (int k = 0; k < 7; ++k) finite = finite && isfinite(q[k]);
  const Acc mu = (Acc)c->mu, tol = (Acc)c->tol, tol_d = (Acc)c->tol_dual;
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
  if (tol > 0 && prel <= tol && drel <= tol_d) {
    c->converged = 1;
    c->done = 1;
  }
  if (c->iter >= c->max_iter) c->done = 1;
}

// Run by one workgroup of kThreads threads; does nothing once the solve has
// stopped.
__device__ __forceinline__ void reduce_in_block(const RedArgs &r) {
  if (r.ctrl->done) return;
  if (r.fp64)
    reduce_body<double, kThreads>(r.ctrl, (const double *)r.ps, r.nbs, (const double *)r.pf, r.nbf);
  else
    reduce_body<float, kThreads>(r.ctrl, (const float *)r.ps, r.nbs, (const float *)r.pf, r.nbf);
}

}  // namespace sr3d
