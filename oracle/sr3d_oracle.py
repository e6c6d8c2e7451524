"""FP64 CPU oracle: 3D-FSR Tikhonov closed form and TV-ADMM (Algorithm 1).

TEST INFRASTRUCTURE ONLY -- imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the HIP library or its binding.

Everything is float64 / complex128, written for a reader holding the paper
(Tuador et al., "A Novel Fast 3D Single Image Super-Resolution Algorithm",
arXiv 2010.15491). Each function names the passage it follows. There is no
blocking, fusion or reordering beyond what the cited formula states; library
primitives used as steps are scipy.fft (unnormalised 3D DFT) and
numpy.linalg.solve.

Conventions (readings of the paper where it is silent, ambiguous or garbled):
  * A volume of size m x n x s (m = rows, fastest in the lexicographic order of
    Sec. II-A and the Kronecker order of eq. (8)) is a C-order array of shape
    (s, n, m).
  * ``rate = (dr, dc, ds)``: dr decimates m, dc decimates n, ds decimates s.
    D keeps the voxel at offset 0 of every dr x dc x ds block.
  * Lambda is the unnormalised 3D DFT of the PSF zero-padded to the HR grid and
    circularly shifted so the PSF's centre voxel (index K//2 per axis) sits at
    index 0 -- i.e. of the first column of the circulant H (eq. (2)).
  * r = d = dr * dc * ds (eq. (9), (12), Algorithm 1 input).
  * L stacks periodic forward differences along m, n, s (component order
    h = m, v = n, s = s); isotropic TV sum_j ||(Lx)_j||_2 (the shrink of
    Algorithm 1 step 5b).
  * Gamma = 1/G is unbounded at the zero frequency (Algorithm 1 step 4); the one
    alias group holding k = 0 is solved as its own d x d linear system.
  * Stopping rule: relative primal/dual residuals (the rule of the ADMM
    reference the paper cites), tested after every iteration.
"""

from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

__all__ = [
    "WORKERS", "hr_shape_of", "lr_shape_of", "psf_to_otf", "blur", "blur_adjoint",
    "decimate", "zero_fill", "degrade", "fold", "unfold", "diff_symbol_sq",
    "grad", "grad_adjoint", "shrink", "shrink_aniso", "tikhonov", "tikhonov_objective",
    "haar3", "haar3_inverse", "haar_detail_mask", "shrink_detail", "wavelet_objective",
    "admm_wavelet", "soft", "l1data_objective", "l1data_residuals", "L1AdmmResult",
    "admm_l1data", "shift", "mf_normal_solve", "tikhonov_mf", "admm_tv_mf", "mf_data_term",
    "gaussian_taps", "separable_blur", "psf_fit_residual", "fit_gaussian_psf",
    "x_update", "AdmmResult", "stopping_residuals", "admm_tv", "min_norm_dual", "tv_objective",
    "data_term", "rel_l2",
]

def _cpu_share():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


WORKERS = _cpu_share()  # scipy.fft threads: this process's CPU share, at most 16


def _fftn(a):
    return sfft.fftn(a, workers=WORKERS)


def _ifftn(a):
    return sfft.ifftn(a, workers=WORKERS)


# ---------------------------------------------------------------------------
# Degradation model, Sec. II-A, eq. (1)-(2)
# ---------------------------------------------------------------------------

def _axes_rate(rate):
    """(dr, dc, ds) -> per-array-axis factors (ds, dc, dr) for shape (s, n, m)."""
    dr, dc, ds = rate
    return (ds, dc, dr)


def hr_shape_of(lr_shape, rate):
    """m_h = m_l*dr, n_h = n_l*dc, s_h = s_l*ds (Sec. II-A)."""
    f = _axes_rate(rate)
    return tuple(int(a) * int(b) for a, b in zip(lr_shape, f))


def lr_shape_of(hr_shape, rate):
    f = _axes_rate(rate)
    for a, b in zip(hr_shape, f):
        if a % b:
            raise ValueError("HR size not divisible by its decimation rate")
    return tuple(int(a) // int(b) for a, b in zip(hr_shape, f))


def psf_to_otf(psf, hr_shape):
    """Lambda of eq. (2): 3D DFT of the zero-padded PSF (first column of H).

    The PSF (shape (Ks, Kn, Km)) is placed in an all-zero HR volume and rolled
    by -(K//2) per axis, so that H is a circular convolution centred on the
    PSF's middle voxel. Unnormalised DFT, as the diagonal of H = F^H Lambda F
    with F unitary.
    """
    psf = np.asarray(psf, dtype=np.float64)
    if any(k > n for k, n in zip(psf.shape, hr_shape)):
        raise ValueError("PSF larger than the volume")
    pad = np.zeros(hr_shape, dtype=np.float64)
    pad[: psf.shape[0], : psf.shape[1], : psf.shape[2]] = psf
    pad = np.roll(pad, shift=tuple(-(k // 2) for k in psf.shape), axis=(0, 1, 2))
    return _fftn(pad)


def blur(x, otf):
    """H x = F^H Lambda F x (eq. (2))."""
    return np.real(_ifftn(otf * _fftn(x)))


def blur_adjoint(x, otf):
    """H^H x = F^H Lambda^H F x (eq. (2))."""
    return np.real(_ifftn(np.conj(otf) * _fftn(x)))


def decimate(z, rate):
    """D: keep one voxel (offset 0) of every dr x dc x ds block."""
    ds, dc, dr = _axes_rate(rate)
    return z[::ds, ::dc, ::dr]


def zero_fill(y, rate):
    """D^H: interpolate with zeros, so that D D^H = I (Sec. II-A)."""
    ds, dc, dr = _axes_rate(rate)
    out = np.zeros(hr_shape_of(y.shape, rate), dtype=np.result_type(y, np.float64))
    out[::ds, ::dc, ::dr] = y
    return out


def degrade(x, psf, rate):
    """Noise-free part of eq. (1): D H x."""
    return decimate(blur(np.asarray(x, np.float64), psf_to_otf(psf, x.shape)), rate)


# ---------------------------------------------------------------------------
# Decimation in the Fourier domain, eq. (8) and the definition of underline-Lambda
# ---------------------------------------------------------------------------

def fold(z, rate):
    """[(1^T (x) I) (x) (1^T (x) I) (x) (1^T (x) I)] z: sum of every alias group.

    An HR spectrum of shape (s_h, n_h, m_h) is viewed as
    (ds, s_l, dc, n_l, dr, m_l); the Kronecker factor 1^T_{ds} (x) I_{s_l} sums
    over the leading ds index, and likewise for n and m.
    """
    ds, dc, dr = _axes_rate(rate)
    S, N, M = z.shape
    v = z.reshape(ds, S // ds, dc, N // dc, dr, M // dr)
    return v.sum(axis=(0, 2, 4))


def unfold(z, rate):
    """Adjoint of ``fold``: replicate an LR-sized array over the alias groups."""
    ds, dc, dr = _axes_rate(rate)
    return np.tile(z, (ds, dc, dr))


# ---------------------------------------------------------------------------
# Finite differences, Sec. III-B and Algorithm 1 steps 3-4
# ---------------------------------------------------------------------------

def diff_symbol_sq(shape):
    """G = Sigma_h^H Sigma_h + Sigma_v^H Sigma_v + Sigma_s^H Sigma_s.

    For a periodic forward difference along an axis of length n the symbol is
    e^{2 pi i k / n} - 1, whose squared modulus is 4 sin^2(pi k / n).
    Gamma of Algorithm 1 step 4 is 1/G (unbounded at k = 0).
    """
    S, N, M = shape
    gs = 4.0 * np.sin(np.pi * np.arange(S) / S) ** 2
    gn = 4.0 * np.sin(np.pi * np.arange(N) / N) ** 2
    gm = 4.0 * np.sin(np.pi * np.arange(M) / M) ** 2
    return gs[:, None, None] + gn[None, :, None] + gm[None, None, :]


def grad(x):
    """L x = [D_h x; D_v x; D_s x]: periodic forward differences.

    Component 0 differences along m (array axis 2), 1 along n (axis 1),
    2 along s (axis 0). (D_a x)[i] = x[i + e_a] - x[i].
    """
    return np.stack([np.roll(x, -1, axis=2) - x,
                     np.roll(x, -1, axis=1) - x,
                     np.roll(x, -1, axis=0) - x])


def grad_adjoint(w):
    """L^T w = sum_a D_a^T w_a with (D_a^T w)[i] = w[i - e_a] - w[i]."""
    return ((np.roll(w[0], 1, axis=2) - w[0])
            + (np.roll(w[1], 1, axis=1) - w[1])
            + (np.roll(w[2], 1, axis=0) - w[2]))


def shrink(nu, thr):
    """Algorithm 1 step 5b: max{0, ||nu_j|| - thr} nu_j / ||nu_j|| per voxel j.

    nu has shape (3, ...); the norm is over the 3 components. Where
    ||nu_j|| = 0 the result is 0.
    """
    nrm = np.sqrt(np.sum(nu * nu, axis=0))
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(nrm > 0, np.maximum(0.0, nrm - thr) / nrm, 0.0)
    return nu * scale[None]


def shrink_aniso(nu, thr):
    """Anisotropic TV, sum_j sum_a |(Lx)_{j,a}|: one of the other regularisers
    the same x-step serves (Sec. III-B). Step 5b becomes the proximal map of
    thr ||.||_1, a soft threshold of every component on its own:
    sign(nu) max{0, |nu| - thr}."""
    return np.sign(nu) * np.maximum(0.0, np.abs(nu) - thr)


# ---------------------------------------------------------------------------
# Tikhonov closed form, Sec. III-A, eq. (5)-(12)
# ---------------------------------------------------------------------------

def tikhonov(y, psf, rate, lam, xbar=None):
    """3D-FSR-l2-l2: the minimiser of eq. (5) through eq. (12).

    k = H^H D^H y + 2 lam xbar, so F k = conj(Lambda) F(D^H y) + 2 lam F xbar.
    x = (1/2lam) k - (1/2lam) F^H Lbar^H (2 lam r I + Lbar Lbar^H)^{-1} Lbar F k,
    where Lbar z = fold(Lambda z), Lbar^H w = conj(Lambda) unfold(w) and
    Lbar Lbar^H = diag(fold(|Lambda|^2)).
    """
    y = np.asarray(y, np.float64)
    hr = hr_shape_of(y.shape, rate)
    otf = psf_to_otf(psf, hr)
    d = int(np.prod(rate))
    Fk = np.conj(otf) * _fftn(zero_fill(y, rate))
    if xbar is not None:
        Fk = Fk + 2.0 * lam * _fftn(np.asarray(xbar, np.float64))
    t = fold(otf * Fk, rate) / (2.0 * lam * d + fold(np.abs(otf) ** 2, rate))
    X = (Fk - np.conj(otf) * unfold(t, rate)) / (2.0 * lam)
    return np.real(_ifftn(X))


def tikhonov_objective(x, y, psf, rate, lam, xbar=None):
    """Eq. (5): 1/2 ||y - D H x||^2 + lam ||x - xbar||^2."""
    r = y - degrade(x, psf, rate)
    dx = x if xbar is None else x - xbar
    return 0.5 * float(np.sum(r * r)) + lam * float(np.sum(dx * dx))


# ---------------------------------------------------------------------------
# TV-ADMM, Sec. III-B, eq. (ADMM), Algorithm 1
# ---------------------------------------------------------------------------

def _dc_group_members(shape, rate):
    """HR indices of the alias group containing k = 0: multiples of the LR size."""
    ds, dc, dr = _axes_rate(rate)
    S, N, M = shape
    sl, nl, ml = S // ds, N // dc, M // dr
    return [(c * sl, b * nl, a * ml)
            for c in range(ds) for b in range(dc) for a in range(dr)]


def x_update(Fk, otf, G, mu, rate):
    """Algorithm 1 step 5a, in the Fourier domain.

    x_f = Gamma Lbar^H (mu r I + Lbar Gamma Lbar^H)^{-1} Lbar Gamma Fk and
    X = (Gamma Fk - x_f) / mu, with Gamma = 1/G.

    Gamma is unbounded at k = 0, so the alias group containing k = 0 is solved
    instead from its own normal equations (the Fourier form of
    (H^T Dbar H + mu L^T L) X = Fk restricted to that group):
        sum_b conj(L_a) L_b X_b / d + mu G_a X_a = Fk_a   for every member a,
    by numpy.linalg.solve. Returns the full HR spectrum X.
    """
    d = int(np.prod(rate))
    with np.errstate(divide="ignore", invalid="ignore"):
        Gam = np.where(G > 0, 1.0 / np.where(G > 0, G, 1.0), 0.0)
    num = fold(otf * Gam * Fk, rate)
    den = mu * d + fold(np.abs(otf) ** 2 * Gam, rate)
    xf = Gam * np.conj(otf) * unfold(num / den, rate)
    X = (Gam * Fk - xf) / mu

    idx = _dc_group_members(Fk.shape, rate)
    lam_v = np.array([otf[i] for i in idx])
    g_v = np.array([G[i] for i in idx])
    b_v = np.array([Fk[i] for i in idx])
    if abs(lam_v[0]) == 0.0:
        raise ZeroDivisionError("Lambda(0) = 0: TV x-update is singular")
    Mdc = np.outer(np.conj(lam_v), lam_v) / d + mu * np.diag(g_v)
    x_v = np.linalg.solve(Mdc, b_v)
    for i, v in zip(idx, x_v):
        X[i] = v
    return X


def data_term(x, y, otf, rate):
    """1/2 ||y - D H x||^2."""
    r = y - decimate(blur(x, otf), rate)
    return 0.5 * float(np.sum(r * r))


def tv_objective(x, y, psf, rate, lam, aniso=False):
    """Eq. (3) with isotropic TV: 1/2||y - DHx||^2 + lam sum_j ||(Lx)_j||_2;
    with ``aniso`` the anisotropic TV lam sum_j ||(Lx)_j||_1."""
    otf = psf_to_otf(psf, x.shape)
    g = grad(x)
    if aniso:
        return data_term(x, y, otf, rate) + lam * float(np.sum(np.abs(g)))
    return data_term(x, y, otf, rate) + lam * float(np.sum(np.sqrt(np.sum(g * g, axis=0))))


@dataclass
class AdmmResult:
    x: np.ndarray
    u: np.ndarray
    d: np.ndarray
    iters: int
    converged: bool
    primal_rel: float
    dual_rel: float
    history: list = field(default_factory=list)


def _rel(num, den):
    return num / den if den > 0 else float("inf")


def stopping_residuals(Kx, u, u_new, d_new, adjoint, mu):
    """Relative primal and dual residuals of the stopping rule.

    Algorithm 1 names a stopping criterion without defining it; the reading
    taken is the relative residuals of the ADMM reference the paper cites
    (primal r = K x - u', dual s = mu K^T (u' - u)) with no absolute term, for
    the split K x = u (K = L for TV, the Haar transform W for the wavelet
    regulariser; ``adjoint`` applies K^T):
        primal = ||K x - u'|| / max(||K x||, ||u'||),
        dual   = mu ||K^T (u' - u)|| / (mu ||K^T d'||).
    A zero denominator gives inf (not converged).
    """
    r_norm = float(np.sqrt(np.sum((Kx - u_new) ** 2)))
    s_norm = mu * float(np.sqrt(np.sum(adjoint(u_new - u) ** 2)))
    pri_den = max(float(np.sqrt(np.sum(Kx * Kx))), float(np.sqrt(np.sum(u_new * u_new))))
    dual_den = mu * float(np.sqrt(np.sum(adjoint(d_new) ** 2)))
    return _rel(r_norm, pri_den), _rel(s_norm, dual_den)


def min_norm_dual(x0, y, psf, rate, mu):
    """Dual warm start (an extension, not in the paper): the minimum-norm d with
    mu L^T d = H^T D^T (y - D H x0) - (its mean), i.e. d = L phi,
    phi = (L^T L)^+ H^T D^T (y - D H x0) / mu (pseudo-inverse: zero mean)."""
    hr = x0.shape
    otf = psf_to_otf(psf, hr)
    r = zero_fill(y - degrade(x0, psf, rate), rate)
    R = np.conj(otf) * _fftn(r)
    G = diff_symbol_sq(hr)
    Phi = np.where(G > 0, R / (mu * np.where(G > 0, G, 1.0)), 0.0)
    return grad(np.real(_ifftn(Phi)))


def admm_tv(y, psf, rate, lam, mu, max_iter, tol=0.0, x0=None, record=False,
            callback=None, warm_dual=False, tol_dual=None, aniso=False):
    """3D-FSR-l2-TV (Algorithm 1). With ``aniso`` the regulariser is the
    anisotropic TV and step 5b the per-component soft threshold
    (``shrink_aniso``); every other step is unchanged.

    Inputs y, H (through ``psf``), lam, r = prod(rate), mu.
    Initialisation: x0 (zero if None); nu = L x0 (with d = 0), u0 = shrink(nu),
    d0 = nu - u0, i.e. steps 5b/5c applied to x0.
    Loop (until the stopping rule holds or ``max_iter`` iterations):
      5a  rho = u - d; Theta = L^T rho; Fk = conj(Lambda) F D^H y + mu F Theta;
          x = F^H X with X from ``x_update``.
      5b  nu = L x + d; u' = shrink(nu, lam/mu).
      5c  d' = d + (L x - u').
    Stopping rule (tol > 0, ``stopping_residuals``): ||L x - u'|| <= tol
    max(||L x||, ||u'||) and mu ||L^T (u' - u)|| <= tol mu ||L^T d'||.
    tol = 0 runs exactly max_iter.
    Output: x of the last x-update (step "Output").
    """
    y = np.asarray(y, np.float64)
    hr = hr_shape_of(y.shape, rate)
    otf = psf_to_otf(psf, hr)
    G = diff_symbol_sq(hr)
    FDty = np.conj(otf) * _fftn(zero_fill(y, rate))
    thr = lam / mu
    prox = shrink_aniso if aniso else shrink

    x = np.zeros(hr) if x0 is None else np.asarray(x0, np.float64).copy()
    nu = grad(x)
    if x0 is not None and warm_dual:
        nu = nu + min_norm_dual(x, y, psf, rate, mu)
    u = prox(nu, thr)
    d = nu - u

    hist = []
    it = 0
    converged = False
    prel = drel = float("inf")
    for it in range(1, max_iter + 1):
        rho = u - d
        theta = grad_adjoint(rho)
        Fk = FDty + mu * _fftn(theta)
        x = np.real(_ifftn(x_update(Fk, otf, G, mu, rate)))
        Lx = grad(x)
        nu = Lx + d
        u_new = prox(nu, thr)
        d_new = d + (Lx - u_new)

        prel, drel = stopping_residuals(Lx, u, u_new, d_new, grad_adjoint, mu)
        if record:
            hist.append((prel, drel))
        if callback is not None:
            callback(it, x, u, d, u_new, d_new)
        u, d = u_new, d_new
        if tol > 0 and prel <= tol and drel <= (tol if not tol_dual else tol_dual):
            converged = True
            break
    return AdmmResult(x=x, u=u, d=d, iters=it, converged=converged,
                      primal_rel=prel, dual_rel=drel, history=hist)


# ---------------------------------------------------------------------------
# l1 in an orthonormal wavelet basis through the same x-step (Sec. III-B):
# phi(W x) = sum of |detail coefficients| of the 3D Haar transform W. With
# W^T W = I the x-step of Algorithm 1 becomes the Tikhonov problem eq. (5)
# with 2 lam -> mu and xbar = W^T (u - d), solved by eq. (12).
# ---------------------------------------------------------------------------

_SQRT_HALF = np.sqrt(0.5)


def _haar_axis(a, axis):
    """(a, b) -> ((a + b)/sqrt 2, (a - b)/sqrt 2) on neighbouring pairs along
    ``axis`` (even index first); its own inverse."""
    a = np.moveaxis(a, axis, 0)
    e, o = a[0::2].copy(), a[1::2].copy()
    a[0::2] = (e + o) * _SQRT_HALF
    a[1::2] = (e - o) * _SQRT_HALF
    return np.moveaxis(a, 0, axis)


def haar3(x, levels=1):
    """W x: the orthonormal 3D Haar transform with ``levels`` levels, in place.

    Level l transforms the previous level's approximation coefficients, which
    sit at the positions that are multiples of 2^(l-1) along every axis: the
    pair map above along m, n and s in turn. Afterwards the approximation
    coefficients sit at the multiples of 2^levels and every other position
    holds a detail coefficient. Every dimension must be a multiple of
    2^levels.
    """
    c = np.array(x, np.float64, copy=True)
    for lev in range(levels):
        st = 2 ** lev
        sub = c[::st, ::st, ::st]
        for axis in (2, 1, 0):
            sub = _haar_axis(sub, axis)
        c[::st, ::st, ::st] = sub
    return c


def haar3_inverse(c, levels=1):
    """W^T c = W^{-1} c (the transform is orthonormal): the levels in reverse."""
    x = np.array(c, np.float64, copy=True)
    for lev in reversed(range(levels)):
        st = 2 ** lev
        sub = x[::st, ::st, ::st]
        for axis in (0, 1, 2):
            sub = _haar_axis(sub, axis)
        x[::st, ::st, ::st] = sub
    return x


def haar_detail_mask(shape, levels=1):
    """True at detail coefficients, False at the approximation ones."""
    st = 2 ** levels
    mask = np.ones(shape, bool)
    mask[::st, ::st, ::st] = False
    return mask


def shrink_detail(nu, thr, mask):
    """Step 5b for phi = thr-weighted l1 of the details: soft threshold where
    ``mask``, identity on the approximation coefficients."""
    return np.where(mask, np.sign(nu) * np.maximum(0.0, np.abs(nu) - thr), nu)


def wavelet_objective(x, y, psf, rate, lam, levels=1):
    """1/2 ||y - D H x||^2 + lam sum |detail coefficients of W x|."""
    otf = psf_to_otf(psf, x.shape)
    c = haar3(x, levels)
    return data_term(x, y, otf, rate) + lam * float(np.sum(np.abs(c[haar_detail_mask(x.shape, levels)])))


def admm_wavelet(y, psf, rate, lam, mu, max_iter, tol=0.0, x0=None, levels=1, record=False,
                 callback=None, tol_dual=None):
    """Algorithm 1 with L replaced by the orthonormal Haar transform W.

    Initialisation as admm_tv: nu = W x0, u = prox(nu), d = nu - u.
    Loop: 5a x = argmin 1/2||y - DHx||^2 + mu/2 ||W x - u + d||^2, i.e.
    ``tikhonov(y, psf, rate, mu/2, xbar=W^T(u - d))``; 5b nu = W x + d,
    u' = shrink_detail(nu, lam/mu); 5c d' = d + (W x - u').
    Stopping rule as admm_tv with L -> W (``stopping_residuals``).
    """
    y = np.asarray(y, np.float64)
    hr = hr_shape_of(y.shape, rate)
    mask = haar_detail_mask(hr, levels)
    thr = lam / mu
    x = np.zeros(hr) if x0 is None else np.asarray(x0, np.float64).copy()
    nu = haar3(x, levels)
    u = shrink_detail(nu, thr, mask)
    d = nu - u
    hist = []
    it = 0
    converged = False
    prel = drel = float("inf")
    for it in range(1, max_iter + 1):
        x = tikhonov(y, psf, rate, 0.5 * mu, xbar=haar3_inverse(u - d, levels))
        c = haar3(x, levels)
        nu = c + d
        u_new = shrink_detail(nu, thr, mask)
        d_new = d + (c - u_new)
        prel, drel = stopping_residuals(c, u, u_new, d_new,
                                        lambda z: haar3_inverse(z, levels), mu)
        if record:
            hist.append((prel, drel))
        if callback is not None:
            callback(it, x, u, d, u_new, d_new)
        u, d = u_new, d_new
        if tol > 0 and prel <= tol and drel <= (tol if not tol_dual else tol_dual):
            converged = True
            break
    return AdmmResult(x=x, u=u, d=d, iters=it, converged=converged,
                      primal_rel=prel, dual_rel=drel, history=hist)


# ---------------------------------------------------------------------------
# Non-Gaussian noise (Sec. V names it as future work): an l1 data term,
#   min_x ||D H x - y||_1 + lam sum_j ||(L x)_j||_2,
# by ADMM with a second split v = D H x - y next to u = L x. The x-step is
# Algorithm 1 step 5a with y -> y + v - e and mu -> mu / mu_data.
# ---------------------------------------------------------------------------

def soft(z, thr):
    """Proximal map of thr ||.||_1: sign(z) max{0, |z| - thr}, elementwise."""
    return np.sign(z) * np.maximum(0.0, np.abs(z) - thr)


def l1data_objective(x, y, psf, rate, lam, aniso=False):
    """||D H x - y||_1 + lam TV(x) (isotropic; anisotropic with ``aniso``)."""
    r = degrade(x, psf, rate) - np.asarray(y, np.float64)
    g = grad(x)
    tv = np.sum(np.abs(g)) if aniso else np.sum(np.sqrt(np.sum(g * g, axis=0)))
    return float(np.sum(np.abs(r))) + lam * float(tv)


def l1data_residuals(t, y, v, v_new, e_new, adjoint_dh, mu_data):
    """Relative residuals of the data split D H x - v = y (the relative
    residuals of the ADMM reference the paper cites, as for the TV split,
    here with a constant c = y on the right-hand side):
        primal = ||D H x - v' - y|| / max(||D H x||, ||v'||, ||y||),
        dual   = mu_data ||(DH)^T (v' - v)|| / (mu_data ||(DH)^T e'||),
    with t = D H x and ``adjoint_dh`` applying H^T D^T. A zero denominator
    gives inf."""
    r_norm = float(np.sqrt(np.sum((t - v_new - y) ** 2)))
    pri_den = max(float(np.sqrt(np.sum(t * t))), float(np.sqrt(np.sum(v_new * v_new))),
                  float(np.sqrt(np.sum(y * y))))
    s_norm = mu_data * float(np.sqrt(np.sum(adjoint_dh(v_new - v) ** 2)))
    dual_den = mu_data * float(np.sqrt(np.sum(adjoint_dh(e_new) ** 2)))
    return _rel(r_norm, pri_den), _rel(s_norm, dual_den)


@dataclass
class L1AdmmResult(AdmmResult):
    v: np.ndarray = None
    e: np.ndarray = None


def admm_l1data(y, psf, rate, lam, mu, mu_data, max_iter, tol=0.0, x0=None, record=False,
                callback=None, tol_dual=None, aniso=False):
    """l1 data term + TV by ADMM with the splits u = L x and v = D H x - y.

    Scaled augmented Lagrangian: ||v||_1 + lam TV(u)
        + mu_data/2 ||D H x - y - v + e||^2 + mu/2 ||L x - u + d||^2.
    Initialisation (steps 5b/5c applied to x0 with zero duals): nu = L x0,
    u = prox(nu, lam/mu), d = nu - u; a = D H x0 - y, v = soft(a, 1/mu_data),
    e = a - v.
    Loop (until the stopping rule holds or ``max_iter`` iterations):
      5a  x = argmin 1/2 ||D H x - (y + v - e)||^2 + (mu/mu_data)/2 ||L x - u + d||^2,
          Algorithm 1 step 5a with y -> y + v - e and mu -> mu/mu_data;
      5b  u' = prox(L x + d, lam/mu); 5c d' = d + L x - u';
      5b' v' = soft(D H x - y + e, 1/mu_data); 5c' e' = e + D H x - y - v'.
    Stopping rule: both splits' relative residuals (``stopping_residuals``
    for u = L x, ``l1data_residuals`` for v = D H x - y); the reported primal
    and dual are the larger of the two splits'. tol = 0 runs max_iter.
    """
    y = np.asarray(y, np.float64)
    hr = hr_shape_of(y.shape, rate)
    otf = psf_to_otf(psf, hr)
    G = diff_symbol_sq(hr)
    thr = lam / mu
    thr_d = 1.0 / mu_data
    mu_r = mu / mu_data
    prox = shrink_aniso if aniso else shrink

    def dh(z):
        return decimate(blur(z, otf), rate)

    def adjoint_dh(z):
        return blur_adjoint(zero_fill(z, rate), otf)

    x = np.zeros(hr) if x0 is None else np.asarray(x0, np.float64).copy()
    nu = grad(x)
    u = prox(nu, thr)
    d = nu - u
    a = dh(x) - y
    v = soft(a, thr_d)
    e = a - v

    hist = []
    it = 0
    converged = False
    prel = drel = float("inf")
    for it in range(1, max_iter + 1):
        Fk = np.conj(otf) * _fftn(zero_fill(y + v - e, rate)) + mu_r * _fftn(grad_adjoint(u - d))
        x = np.real(_ifftn(x_update(Fk, otf, G, mu_r, rate)))
        Lx = grad(x)
        u_new = prox(Lx + d, thr)
        d_new = d + (Lx - u_new)
        t = dh(x)
        v_new = soft(t - y + e, thr_d)
        e_new = e + (t - y - v_new)

        p_tv, d_tv = stopping_residuals(Lx, u, u_new, d_new, grad_adjoint, mu)
        p_da, d_da = l1data_residuals(t, y, v, v_new, e_new, adjoint_dh, mu_data)
        prel, drel = max(p_tv, p_da), max(d_tv, d_da)
        if record:
            hist.append((prel, drel, p_tv, d_tv, p_da, d_da))
        if callback is not None:
            callback(it, x, u, d, u_new, d_new, v, e, v_new, e_new)
        u, d, v, e = u_new, d_new, v_new, e_new
        if tol > 0 and prel <= tol and drel <= (tol if not tol_dual else tol_dual):
            converged = True
            break
    return L1AdmmResult(x=x, u=u, d=d, iters=it, converged=converged, primal_rel=prel,
                        dual_rel=drel, history=hist, v=v, e=e)


# ---------------------------------------------------------------------------
# 3D multi-frame SR (Sec. V names it as future work): F LR frames
# y_f = D S_f H x + n_f of one HR volume, S_f a known circular shift of the HR
# grid by t_f = (t_m, t_n, t_s) voxels, (S_f z)[i] = z[i + t_f]. With
# F(S_f z)_k = w_f(k) Z_k, w_f(k) = exp(+2 pi i k . t_f / n), eq. (8) gives
# F_LR(y_f)_j = (1/d) sum_a w_f(k_a) Lambda_a X_a over the alias group of j,
# so the normal equations still split into one d x d system per group, now
# with F rank-one terms:
#   sum_f conj(v_f) (1/d) v_f^T X + diag(A) X = B,  v_f = w_f Lambda,
#   B_a = sum_f conj(v_f,a) F_LR(y_f)_j + c W_a.
# ---------------------------------------------------------------------------

def shift(z, t):
    """S z with (S z)[i] = z[i + t] (circular), t = (t_m, t_n, t_s)."""
    return np.roll(z, shift=(-int(t[2]), -int(t[1]), -int(t[0])), axis=(0, 1, 2))


def _mf_phase(shape, t):
    """w(k) = exp(2 pi i (k_m t_m / M + k_n t_n / N + k_s t_s / S))."""
    S, N, M = shape
    ps = np.exp(2j * np.pi * np.arange(S) * t[2] / S)
    pn = np.exp(2j * np.pi * np.arange(N) * t[1] / N)
    pm = np.exp(2j * np.pi * np.arange(M) * t[0] / M)
    return ps[:, None, None] * pn[None, :, None] * pm[None, None, :]


def _groups(z, rate):
    """HR spectrum (S, N, M) -> (S_l, N_l, M_l, d) member arrays, members in
    the order (c, b, a) of the alias offsets (c along s, b along n, a along m)."""
    ds, dc, dr = _axes_rate(rate)
    S, N, M = z.shape
    v = z.reshape(ds, S // ds, dc, N // dc, dr, M // dr)
    return v.transpose(1, 3, 5, 0, 2, 4).reshape(S // ds, N // dc, M // dr, ds * dc * dr)


def _ungroups(g, rate, shape):
    ds, dc, dr = _axes_rate(rate)
    S, N, M = shape
    v = g.reshape(S // ds, N // dc, M // dr, ds, dc, dr).transpose(3, 0, 4, 1, 5, 2)
    return v.reshape(shape)


def mf_normal_solve(Yf, otf, phases, A, W, c, rate):
    """Per alias group, numpy.linalg.solve of
    (sum_f conj(v_f) (1/d) v_f^T + diag(A)) X = B,  v_f = phase_f Lambda,
    B = sum_f conj(v_f) Y_f[j] + c W (W may be None). Yf: list of LR spectra
    (full, complex); returns the HR spectrum X."""
    d = int(np.prod(rate))
    shape = otf.shape
    V = [_groups(ph * otf, rate) for ph in phases]          # (..., d) each
    Ag = _groups(np.broadcast_to(A, shape).astype(complex), rate)
    K = np.zeros(Ag.shape + (d,), complex)
    B = np.zeros(Ag.shape, complex)
    for v, y in zip(V, Yf):
        K += np.conj(v)[..., :, None] * v[..., None, :] / d
        B += np.conj(v) * y[..., None]
    K += Ag[..., :, None] * np.eye(d)
    if W is not None:
        B += c * _groups(W, rate)
    X = np.linalg.solve(K, B[..., None])[..., 0]
    return _ungroups(X, rate, shape)


def tikhonov_mf(ys, shifts, psf, rate, lam, xbar=None):
    """Multi-frame eq. (5): min sum_f 1/2 ||y_f - D S_f H x||^2 + lam ||x - xbar||^2,
    solved per alias group (A = 2 lam, c = 2 lam, W = F xbar)."""
    ys = [np.asarray(y, np.float64) for y in ys]
    hr = hr_shape_of(ys[0].shape, rate)
    otf = psf_to_otf(psf, hr)
    phases = [_mf_phase(hr, t) for t in shifts]
    Yf = [_fftn(y) for y in ys]
    W = None if xbar is None else _fftn(np.asarray(xbar, np.float64))
    X = mf_normal_solve(Yf, otf, phases, np.full(hr, 2.0 * lam), W, 2.0 * lam, rate)
    return np.real(_ifftn(X))


def mf_data_term(x, ys, shifts, psf, rate):
    """sum_f 1/2 ||y_f - D S_f H x||^2."""
    otf = psf_to_otf(psf, x.shape)
    hx = blur(x, otf)
    return 0.5 * sum(float(np.sum((np.asarray(y) - decimate(shift(hx, t), rate)) ** 2))
                     for y, t in zip(ys, shifts))


def admm_tv_mf(ys, shifts, psf, rate, lam, mu, max_iter, tol=0.0, x0=None, record=False,
               callback=None, aniso=False):
    """Algorithm 1 with the multi-frame data term: step 5a is the multi-frame
    normal equations (A = mu G, c = mu, W = F Theta) solved per group;
    steps 5b/5c and the stopping rule are unchanged."""
    ys = [np.asarray(y, np.float64) for y in ys]
    hr = hr_shape_of(ys[0].shape, rate)
    otf = psf_to_otf(psf, hr)
    G = diff_symbol_sq(hr)
    phases = [_mf_phase(hr, t) for t in shifts]
    Yf = [_fftn(y) for y in ys]
    thr = lam / mu
    prox = shrink_aniso if aniso else shrink
    x = np.zeros(hr) if x0 is None else np.asarray(x0, np.float64).copy()
    nu = grad(x)
    u = prox(nu, thr)
    d = nu - u
    hist = []
    it = 0
    converged = False
    prel = drel = float("inf")
    for it in range(1, max_iter + 1):
        theta = grad_adjoint(u - d)
        X = mf_normal_solve(Yf, otf, phases, mu * G, _fftn(theta), mu, rate)
        x = np.real(_ifftn(X))
        Lx = grad(x)
        u_new = prox(Lx + d, thr)
        d_new = d + (Lx - u_new)
        prel, drel = stopping_residuals(Lx, u, u_new, d_new, grad_adjoint, mu)
        if record:
            hist.append((prel, drel))
        if callback is not None:
            callback(it, x, u, d, u_new, d_new)
        u, d = u_new, d_new
        if tol > 0 and prel <= tol and drel <= tol:
            converged = True
            break
    return AdmmResult(x=x, u=u, d=d, iters=it, converged=converged,
                      primal_rel=prel, dual_rel=drel, history=hist)


# ---------------------------------------------------------------------------
# PSF estimation (Sec. IV-B): the PSF of the real data is estimated by fitting
# a 3D Gaussian; the paper reports only the fitted widths. Reading: the HR
# reference x (the micro-CT, registered to the CBCT grid) and the LR volume y
# are given, and sigma = (sigma_m, sigma_n, sigma_s) of a separable, sampled,
# normalised Gaussian on a fixed support, with an intensity gain alpha and
# offset beta, minimises 1/2 ||y - alpha D H_sigma x - beta||^2.
# ---------------------------------------------------------------------------

def gaussian_taps(sigma, radius):
    """g[i] = exp(-i^2 / (2 sigma^2)) / sum, i = -radius..radius."""
    i = np.arange(-int(radius), int(radius) + 1, dtype=np.float64)
    g = np.exp(-(i * i) / (2.0 * float(sigma) ** 2))
    return g / g.sum()


def separable_blur(x, sigma, radius):
    """H_sigma x in the spatial domain: circular convolution with
    gaussian_taps along m, n and s in turn (``sigma``, ``radius`` as
    (m, n, s)); the kernel is symmetric, so convolution = correlation."""
    from scipy import ndimage
    out = np.asarray(x, np.float64)
    for axis, sg, r in ((2, sigma[0], radius[0]), (1, sigma[1], radius[1]),
                        (0, sigma[2], radius[2])):
        out = ndimage.correlate1d(out, gaussian_taps(sg, r), axis=axis, mode="wrap")
    return out


def psf_fit_residual(theta, x, y, rate, radius):
    """y - alpha D H_sigma x - beta for theta = (sigma_m, sigma_n, sigma_s,
    alpha, beta), flattened."""
    sm, sn, ss, alpha, beta = (float(t) for t in theta)
    model = decimate(separable_blur(x, (sm, sn, ss), radius), rate)
    return (np.asarray(y, np.float64) - alpha * model - beta).ravel()


def fit_gaussian_psf(x, y, rate, sigma0, radius, alpha0=1.0, beta0=0.0):
    """Least-squares fit of (sigma, alpha, beta) by scipy's trust-region
    solver (numerical Jacobian), from sigma0. Returns (sigma, alpha, beta,
    1/2 ||residual||^2)."""
    from scipy.optimize import least_squares
    th0 = np.array(list(sigma0) + [alpha0, beta0], np.float64)
    lo = np.array([0.05, 0.05, 0.05, -np.inf, -np.inf])
    res = least_squares(psf_fit_residual, th0, args=(x, y, rate, radius), bounds=(lo, np.inf),
                        method="trf", x_scale="jac", xtol=1e-14, ftol=1e-14, gtol=1e-14,
                        max_nfev=500)
    th = res.x
    return tuple(th[:3]), float(th[3]), float(th[4]), 0.5 * float(np.sum(res.fun ** 2))


# ---------------------------------------------------------------------------
# Metrics
# ---------------------------------------------------------------------------

def rel_l2(a, b):
    """||a - b|| / ||b|| in float64."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = float(np.linalg.norm(b.ravel()))
    return float(np.linalg.norm((a - b).ravel())) / (nb if nb > 0 else 1.0)
