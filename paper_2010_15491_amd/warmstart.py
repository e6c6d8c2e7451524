"""Learned warm start for TV-ADMM: training pairs, training loop, inference.

Host-side sequencing only: every numerical step is a libsr3d call (forward
model, Tikhonov closed form, batched TV-ADMM, CNN gradient, Adam, CNN
forward). Inputs are seeded synthetic ellipsoid phantoms.
"""

from __future__ import annotations

import time
from dataclasses import dataclass

from . import phantom, sr3d


def make_pairs(seeds, shape=(64, 64, 64), rate=(2, 2, 2), sigma=1.5, noise=0.02, tau=1e-3,
               lam=2e-3, mu=5e-2, tol=1e-4, cap=200, chunk=64, device="cuda"):
    """(Tikhonov solution, plain TV-ADMM solution) for each seed.

    The plain solutions come from sr3d_batch in chunks of `chunk` volumes.
    Returns a list of (x_tik, x_admm) device tensors and the ADMM stats.
    """
    import torch
    pairs, stats = [], []
    seeds = list(seeds)
    for c0 in range(0, len(seeds), chunk):
        probs, tiks = [], []
        for seed in seeds[c0:c0 + chunk]:
            p = phantom.make_problem(shape, rate, sigma, noise, seed)
            psf = torch.from_numpy(p["psf"].astype("float32")).to(device)
            xt = torch.from_numpy(p["x_true"].astype("float32")).to(device)
            y = sr3d.degrade(xt, psf, rate)
            y += torch.from_numpy(p["noise"].astype("float32")).to(device)
            tiks.append(sr3d.tikhonov(y, psf, rate, tau))
            probs.append(dict(y=y, psf=psf, rate=rate, lam=lam, mu=mu, tol=tol, max_iter=cap))
        xs, sts = sr3d.batch(probs)
        pairs += list(zip(tiks, xs))
        stats += sts
    return pairs, stats


def train(pairs, steps, lr=1e-3, lr_final=1e-4, seed=0, log_every=0):
    """Adam on the mean squared error between x_tik + f(x_tik) and x_admm,
    one pair per step, cycling through the pairs in a seeded random order;
    the learning rate decays geometrically from lr to lr_final.
    Returns (params, list of (step, loss))."""
    import numpy as np
    import torch
    params = sr3d.cnn_init(seed)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    ws = sr3d.CnnWorkspace(pairs[0][0].shape)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    rng = np.random.default_rng(seed)
    order = rng.permutation(len(pairs))
    hist = []
    losses = torch.empty(steps, dtype=torch.float32, device=params.device)
    for step in range(1, steps + 1):
        i = order[(step - 1) % len(pairs)]
        if step % len(pairs) == 0:
            order = rng.permutation(len(pairs))
        xt, xa = pairs[i]
        sr3d.cnn_grad(params, xt, xa, grad=grad, loss=loss, ws=ws)
        rate = lr * (lr_final / lr) ** ((step - 1) / max(steps - 1, 1))
        sr3d.cnn_adam(params, grad, m, v, step, rate)
        losses[step - 1] = loss[0]
        if log_every and step % log_every == 0:
            hist.append((step, float(losses[step - 1].item())))
    torch.cuda.synchronize()
    return params, losses.cpu().tolist(), hist


def warm_start(params, y, psf, rate, tau=1e-3, ws=None):
    """x0 = x_tik + f(x_tik) with x_tik the Tikhonov solution (eq. (12))."""
    xt = sr3d.tikhonov(y, psf, rate, tau)
    return sr3d.cnn_forward(params, xt, ws=ws)


@dataclass
class WarmSolve:
    """Outcome of solve(): which start produced x, and the stats of each run."""
    used: str                      # "warm" (accepted) or "plain" (fallback)
    warm: sr3d.AdmmStats           # the run from the learned x0
    plain: sr3d.AdmmStats | None   # the fallback run from x0 = 0, if it ran


def solve(params, y, psf, rate, lam, mu, max_iter, tol, tol_dual=0.0, tau=1e-3, out=None,
          workspace=None, cnn_ws=None, flags=sr3d.FP64_REDUCE):
    """Algorithm 1 from the learned start, with plain ADMM as the fallback.

    x0 = x_tik + f(x_tik) starts a TV-ADMM solve to `tol` (cap `max_iter`).
    The result is accepted only if that solve meets the tolerance (both
    relative residuals); otherwise plain ADMM from x0 = 0 runs to the same
    tolerance and cap and its x is returned, so a caller always gets what the
    method without the network gives unless the warm start has converged.
    Both runs' time is paid. Returns (x, WarmSolve)."""
    x0 = warm_start(params, y, psf, rate, tau, ws=cnn_ws)
    x, stw = sr3d.tv_admm(y, psf, rate, lam, mu, max_iter, tol=tol, tol_dual=tol_dual, x0=x0,
                          flags=flags, out=out, workspace=workspace)
    if stw.converged:
        return x, WarmSolve("warm", stw, None)
    x, stp = sr3d.tv_admm(y, psf, rate, lam, mu, max_iter, tol=tol, tol_dual=tol_dual,
                          flags=flags, out=x, workspace=workspace)
    return x, WarmSolve("plain", stw, stp)


def timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0
