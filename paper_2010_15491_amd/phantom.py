"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module draws random numbers and samples a Gaussian PSF; it holds none of
the solver's arithmetic (no blur, decimation, FFT-domain solve or ADMM step).
The measurement y = D H x + n is formed by whichever side consumes these inputs
(the oracle's ``degrade`` in tests, the library's ``sr3d_degrade`` in the
benchmark), each with its own code.

Arrays are C-order (s, n, m): m (rows) is the fastest axis. A PSF size or
sigma is given as (m, n, s) like the volume dimensions in the paper's notation.

Recipe (the paper's tooth scans are not available; these phantoms stand in):
  * ellipsoid phantom: ``rng = numpy.random.default_rng(seed)``; voxel-centre
    coordinates t in (0,1)^3; for each of 12 ellipsoids, in this draw order:
    centre c ~ U[0.2,0.8]^3, semi-axes a ~ U[0.05,0.25]^3, rotation Q from the
    QR factorisation of a 3x3 N(0,1) matrix with column signs fixed by diag(R),
    intensity v ~ U[0,1]; x += v * [ ||Q^T (t - c) / a|| <= 1 ].
  * optional smooth texture: HR N(0,1) white noise, circular Gaussian smoothing
    with sigma_t = 4 voxels (scipy.ndimage, mode "wrap"), rescaled to std 0.05,
    added to x.
  * noise: sigma_n * N(0,1) on the LR grid, drawn after phantom and texture.
  * PSF: separable sampled Gaussian exp(-i^2 / (2 sigma^2)) at integer offsets
    i in [-K//2, K//2], K = 2*ceil(2 sigma) + 1 per axis, normalised to sum 1.
  * impulse noise (the non-Gaussian noise an l1 data term is for):
    ``default_rng(seed)``; each LR voxel is hit with probability ``frac``
    (uniform draw < frac), then gets +amp or -amp with equal probability;
    added to the Gaussian noise above.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = ["psf_size", "gaussian_psf", "ellipsoid_phantom", "texture_field",
           "make_problem", "lr_shape", "impulse_noise"]


def psf_size(sigma):
    """K = 2*ceil(2 sigma) + 1."""
    return 2 * int(math.ceil(2.0 * float(sigma) - 1e-12)) + 1


def gaussian_psf(sigma):
    """Sampled, normalised 3D Gaussian. ``sigma`` is a scalar or (sm, sn, ss).

    Returns shape (Ks, Kn, Km), float64, summing to 1.
    """
    if np.isscalar(sigma):
        sigma = (sigma, sigma, sigma)
    sm, sn, ss = (float(v) for v in sigma)
    axes = []
    for sg in (ss, sn, sm):
        k = psf_size(sg)
        i = np.arange(k) - k // 2
        axes.append(np.exp(-(i * i) / (2.0 * sg * sg)))
    p = axes[0][:, None, None] * axes[1][None, :, None] * axes[2][None, None, :]
    return p / p.sum()


def ellipsoid_phantom(shape, rng, n_ellipsoids=12):
    """Sum of ``n_ellipsoids`` random solid ellipsoids on a (s, n, m) grid."""
    S, N, M = shape
    x = np.zeros(shape, dtype=np.float64)
    dims = np.array([M, N, S], dtype=np.float64)  # coordinate order (m, n, s)
    for _ in range(n_ellipsoids):
        c = rng.uniform(0.2, 0.8, 3)
        a = rng.uniform(0.05, 0.25, 3)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        v = rng.uniform(0.0, 1.0)
        # Bounding box of the rotated ellipsoid: half-extent along axis i is
        # sqrt(sum_k (Q_ik a_k)^2). Only voxels inside it can satisfy the test.
        ext = np.sqrt(np.sum((q * a[None, :]) ** 2, axis=1))
        lo = np.floor((c - ext) * dims - 0.5).astype(int)
        hi = np.ceil((c + ext) * dims - 0.5).astype(int) + 1
        lo = np.clip(lo, 0, dims.astype(int))
        hi = np.clip(hi, 0, dims.astype(int))
        if np.any(hi <= lo):
            continue
        tm = (np.arange(lo[0], hi[0]) + 0.5) / M - c[0]
        tn = (np.arange(lo[1], hi[1]) + 0.5) / N - c[1]
        ts = (np.arange(lo[2], hi[2]) + 0.5) / S - c[2]
        # p = (tm, tn, ts); z = Q^T p / a ; inside if |z| <= 1
        acc = np.zeros((len(ts), len(tn), len(tm)))
        for k in range(3):
            zk = (q[0, k] * tm[None, None, :] + q[1, k] * tn[None, :, None]
                  + q[2, k] * ts[:, None, None]) / a[k]
            acc += zk * zk
        x[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += v * (acc <= 1.0)
    return x


def texture_field(shape, rng, sigma_t=4.0, std=0.05):
    """Smooth-texture noise: Gaussian-smoothed white noise rescaled to ``std``."""
    from scipy import ndimage

    w = rng.standard_normal(shape)
    sm = ndimage.gaussian_filter(w, sigma=sigma_t, mode="wrap")
    s = float(np.std(sm))
    return sm * (std / s) if s > 0 else sm


def lr_shape(hr_shape, rate):
    """LR shape (s_l, n_l, m_l) for HR shape (s, n, m) and rate (dr, dc, ds)."""
    S, N, M = hr_shape
    dr, dc, ds = rate
    if S % ds or N % dc or M % dr:
        raise ValueError("HR size not divisible by its decimation rate")
    return (S // ds, N // dc, M // dr)


def make_problem(hr_shape, rate, sigma, noise_sigma, seed, texture=False,
                 n_ellipsoids=12):
    """Seeded phantom, PSF and LR noise for one problem.

    Returns dict with ``x_true`` (HR float64), ``psf`` (float64),
    ``noise`` (LR float64, already scaled by ``noise_sigma``), ``rate``.
    """
    rng = np.random.default_rng(seed)
    x = ellipsoid_phantom(hr_shape, rng, n_ellipsoids)
    if texture:
        x = x + texture_field(hr_shape, rng)
    noise = noise_sigma * rng.standard_normal(lr_shape(hr_shape, rate))
    return {"x_true": x, "psf": gaussian_psf(sigma), "noise": noise,
            "rate": tuple(rate)}


def impulse_noise(shape, seed, frac=0.1, amp=1.0):
    """Sparse +-amp impulses on a fraction ``frac`` of the voxels of ``shape``."""
    rng = np.random.default_rng(seed)
    hit = rng.random(shape) < frac
    sign = np.where(rng.random(shape) < 0.5, -1.0, 1.0)
    return hit * sign * float(amp)
