"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something it does not share code with:
brute-force sums and dense matrices built voxel by voxel, scipy.ndimage's
circular convolution, closed forms of special cases, optimality (KKT)
conditions of the convex problems, and invariants of the ADMM iteration.
The paper prints no worked numeric example (its data are private scans), so
there is no printed value to pin against.
"""

import numpy as np
import pytest
from scipy import ndimage

import oracle as O

# ---------------------------------------------------------------------------
# Independent spatial-domain operators (no FFT), used only by the pins
# ---------------------------------------------------------------------------


def conv_wrap(x, psf):
    """H x as a circular convolution centred on the PSF's middle voxel."""
    return ndimage.convolve(x, psf, mode="wrap")


def corr_wrap(x, psf):
    """H^T x: circular correlation with the same centring."""
    return ndimage.correlate(x, psf, mode="wrap")


def dense_H(psf, shape):
    """Dense circulant H: (H x)[i] = sum_p psf[p] x[i - (p - K//2)] (mod shape)."""
    S, N, M = shape
    n = S * N * M
    idx = np.arange(n).reshape(shape)
    H = np.zeros((n, n))
    Ks, Kn, Km = psf.shape
    for ps in range(Ks):
        for pn in range(Kn):
            for pm in range(Km):
                src = np.roll(idx, shift=(ps - Ks // 2, pn - Kn // 2, pm - Km // 2),
                              axis=(0, 1, 2))
                H[idx.ravel(), src.ravel()] += psf[ps, pn, pm]
    return H


def dense_D(shape, rate):
    """Dense decimation: keeps voxel (0,0,0) of every ds x dc x dr block."""
    dr, dc, ds = rate
    S, N, M = shape
    keep = [(s * N + n) * M + m
            for s in range(0, S, ds) for n in range(0, N, dc) for m in range(0, M, dr)]
    D = np.zeros((len(keep), S * N * M))
    D[np.arange(len(keep)), keep] = 1.0
    return D


def dense_L(shape):
    """Dense L (3N x N): periodic forward differences along m, n, s."""
    S, N, M = shape
    n = S * N * M
    L = np.zeros((3 * n, n))
    for s in range(S):
        for q in range(N):
            for m in range(M):
                i = (s * N + q) * M + m
                nb = [(s * N + q) * M + (m + 1) % M,
                      (s * N + (q + 1) % N) * M + m,
                      (((s + 1) % S) * N + q) * M + m]
                for a in range(3):
                    L[a * n + i, nb[a]] += 1.0
                    L[a * n + i, i] -= 1.0
    return L


def rand_psf(rng, shape):
    p = rng.uniform(0.05, 1.0, shape)
    return p / p.sum()


# ---------------------------------------------------------------------------
# Eq. (2): Lambda diagonalises the circulant blur
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,kshape", [((6, 7, 8), (3, 2, 5)), ((4, 4, 4), (3, 3, 3)),
                                          ((8, 6, 9), (5, 1, 4))])
def test_otf_is_bruteforce_dft_of_first_column(shape, kshape):
    rng = np.random.default_rng(1)
    psf = rand_psf(rng, kshape)
    H = dense_H(psf, shape)
    col = H[:, 0].reshape(shape)
    S, N, M = shape
    ks, kn, km = np.meshgrid(np.arange(S), np.arange(N), np.arange(M), indexing="ij")
    lam = np.zeros(shape, complex)
    for s in range(S):
        for q in range(N):
            for m in range(M):
                lam += col[s, q, m] * np.exp(-2j * np.pi * (ks * s / S + kn * q / N + km * m / M))
    assert np.allclose(O.psf_to_otf(psf, shape), lam, atol=1e-13)


@pytest.mark.parametrize("shape,kshape", [((16, 12, 8), (5, 3, 4)), ((9, 8, 12), (7, 7, 7))])
def test_blur_and_adjoint_match_ndimage(shape, kshape):
    rng = np.random.default_rng(2)
    psf = rand_psf(rng, kshape)
    x = rng.standard_normal(shape)
    otf = O.psf_to_otf(psf, shape)
    assert np.allclose(O.blur(x, otf), conv_wrap(x, psf), atol=1e-13)
    assert np.allclose(O.blur_adjoint(x, otf), corr_wrap(x, psf), atol=1e-13)


def test_degrade_matches_dense():
    rng = np.random.default_rng(3)
    shape, rate = (4, 6, 8), (2, 3, 2)
    psf = rand_psf(rng, (3, 3, 2))
    x = rng.standard_normal(shape)
    y = dense_D(shape, rate) @ dense_H(psf, shape) @ x.ravel()
    assert np.allclose(O.degrade(x, psf, rate).ravel(), y, atol=1e-13)


# ---------------------------------------------------------------------------
# Eq. (8): decimation in the Fourier domain
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,rate", [((8, 8, 8), (2, 2, 2)), ((8, 9, 6), (2, 3, 4)),
                                        ((4, 8, 16), (4, 4, 2)), ((6, 4, 8), (1, 2, 3))])
def test_fold_identity_eq8(shape, rate):
    """F (D^H D) F^H = alias-group mean, replicated over the group."""
    rng = np.random.default_rng(4)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d = int(np.prod(rate))
    mask = np.zeros(shape)
    dr, dc, ds = rate
    mask[::ds, ::dc, ::dr] = 1.0
    lhs = np.fft.fftn(mask * np.fft.ifftn(z))
    rhs = O.unfold(O.fold(z, rate), rate) / d
    assert np.allclose(lhs, rhs, atol=1e-12)


def test_fold_unfold_are_adjoint():
    rng = np.random.default_rng(5)
    shape, rate = (8, 6, 12), (3, 2, 4)
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    w = rng.standard_normal(O.lr_shape_of(shape, rate)) + 1j * rng.standard_normal(
        O.lr_shape_of(shape, rate))
    lhs = np.vdot(w, O.fold(z, rate))
    rhs = np.vdot(O.unfold(w, rate), z)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_zero_fill_fft_is_replicated_lr_fft():
    """F D^H y is the LR DFT of y replicated over the alias groups."""
    rng = np.random.default_rng(6)
    rate = (2, 2, 4)
    y = rng.standard_normal((3, 5, 4))
    lhs = np.fft.fftn(O.zero_fill(y, rate))
    assert np.allclose(lhs, O.unfold(np.fft.fftn(y), rate), atol=1e-12)


# ---------------------------------------------------------------------------
# Eq. (5)-(12): Tikhonov closed form
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,rate,kshape", [((8, 8, 8), (2, 2, 2), (3, 3, 3)),
                                               ((4, 6, 8), (2, 3, 2), (3, 2, 5)),
                                               ((8, 4, 4), (1, 2, 4), (2, 3, 3)),
                                               ((4, 4, 8), (4, 1, 1), (1, 1, 5))])
def test_tikhonov_matches_dense_eq6(shape, rate, kshape):
    rng = np.random.default_rng(7)
    psf = rand_psf(rng, kshape)
    lam = 0.013
    lr = O.lr_shape_of(shape, rate)
    y = rng.standard_normal(lr)
    xbar = rng.standard_normal(shape)
    H = dense_H(psf, shape)
    D = dense_D(shape, rate)
    n = H.shape[0]
    A = H.T @ D.T @ D @ H + 2 * lam * np.eye(n)
    b = H.T @ D.T @ y.ravel() + 2 * lam * xbar.ravel()
    x_dense = np.linalg.solve(A, b).reshape(shape)
    x = O.tikhonov(y, psf, rate, lam, xbar)
    assert np.abs(x - x_dense).max() < 1e-10 * max(1.0, np.abs(x_dense).max())
    x0 = O.tikhonov(y, psf, rate, lam, None)
    x0_dense = np.linalg.solve(A, H.T @ D.T @ y.ravel()).reshape(shape)
    assert np.allclose(x0, x0_dense, atol=1e-10)


def test_tikhonov_rate_one_is_wiener():
    """d = 1: X = (conj(L) Y + 2 lam Xbar) / (|L|^2 + 2 lam), classic deconvolution."""
    rng = np.random.default_rng(8)
    shape = (8, 12, 16)
    psf = rand_psf(rng, (5, 3, 3))
    y = rng.standard_normal(shape)
    xbar = rng.standard_normal(shape)
    lam = 0.05
    L = np.fft.fftn(np.roll(np.pad(psf, [(0, s - k) for s, k in zip(shape, psf.shape)]),
                            (-2, -1, -1), axis=(0, 1, 2)))
    X = (np.conj(L) * np.fft.fftn(y) + 2 * lam * np.fft.fftn(xbar)) / (np.abs(L) ** 2 + 2 * lam)
    assert np.allclose(O.tikhonov(y, psf, (1, 1, 1), lam, xbar), np.real(np.fft.ifftn(X)),
                       atol=1e-12)


def test_tikhonov_delta_psf_spatial_closed_form():
    """H = I: x = (y + 2 lam xbar)/(1 + 2 lam) on kept voxels, xbar elsewhere."""
    rng = np.random.default_rng(9)
    shape, rate = (8, 12, 8), (2, 3, 4)
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    xbar = rng.standard_normal(shape)
    lam = 0.2
    x = O.tikhonov(y, np.ones((1, 1, 1)), rate, lam, xbar)
    ref = xbar.copy()
    dr, dc, ds = rate
    ref[::ds, ::dc, ::dr] = (y + 2 * lam * xbar[::ds, ::dc, ::dr]) / (1 + 2 * lam)
    assert np.allclose(x, ref, atol=1e-12)


def test_tikhonov_gradient_vanishes_at_32cube():
    """Eq. (5) optimality at a BASELINE-shaped problem, with spatial operators."""
    from paper_2010_15491_amd import phantom
    p = phantom.make_problem((32, 32, 32), (2, 2, 2), 1.0, 0.01, 0)
    y = O.degrade(p["x_true"], p["psf"], p["rate"]) + p["noise"]
    lam = 1e-3
    x = O.tikhonov(y, p["psf"], p["rate"], lam)
    r = O.zero_fill(O.decimate(conv_wrap(x, p["psf"]), p["rate"]) - y, p["rate"])
    g = corr_wrap(r, p["psf"]) + 2 * lam * x
    scale = np.abs(corr_wrap(O.zero_fill(y, p["rate"]), p["psf"])).max()
    assert np.abs(g).max() < 1e-11 * scale


def test_tikhonov_is_minimum_of_eq5():
    rng = np.random.default_rng(10)
    shape, rate = (8, 8, 16), (2, 2, 2)
    psf = rand_psf(rng, (3, 3, 3))
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    lam = 0.01
    x = O.tikhonov(y, psf, rate, lam)
    f0 = O.tikhonov_objective(x, y, psf, rate, lam)
    for _ in range(5):
        v = rng.standard_normal(shape)
        assert O.tikhonov_objective(x + 1e-3 * v, y, psf, rate, lam) > f0


# ---------------------------------------------------------------------------
# Algorithm 1: x-update, shrink, invariants, KKT
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,rate,kshape", [((8, 8, 8), (2, 2, 2), (3, 3, 3)),
                                               ((4, 8, 8), (2, 2, 4), (3, 3, 2)),
                                               ((8, 8, 4), (4, 4, 2), (3, 2, 3)),
                                               ((6, 4, 8), (2, 1, 3), (1, 3, 5))])
def test_x_update_matches_dense_normal_equations(shape, rate, kshape):
    """Step 5a = argmin 1/2||y-DHx||^2 + mu/2||Lx-rho||^2, including the DC group."""
    rng = np.random.default_rng(11)
    psf = rand_psf(rng, kshape)
    mu = 0.07
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    rho = rng.standard_normal((3,) + shape)
    H, D, L = dense_H(psf, shape), dense_D(shape, rate), dense_L(shape)
    A = H.T @ D.T @ D @ H + mu * L.T @ L
    b = H.T @ D.T @ y.ravel() + mu * L.T @ rho.reshape(-1)
    x_dense = np.linalg.solve(A, b).reshape(shape)
    otf = O.psf_to_otf(psf, shape)
    Fk = np.conj(otf) * np.fft.fftn(O.zero_fill(y, rate)) + mu * np.fft.fftn(O.grad_adjoint(rho))
    x = np.real(np.fft.ifftn(O.x_update(Fk, otf, O.diff_symbol_sq(shape), mu, rate)))
    assert np.abs(x - x_dense).max() < 1e-10 * np.abs(x_dense).max()


def test_grad_and_adjoint_match_dense_L():
    rng = np.random.default_rng(12)
    shape = (4, 5, 6)
    L = dense_L(shape)
    x = rng.standard_normal(shape)
    w = rng.standard_normal((3,) + shape)
    assert np.allclose(O.grad(x).reshape(-1), L @ x.ravel(), atol=1e-14)
    assert np.allclose(O.grad_adjoint(w).ravel(), L.T @ w.reshape(-1), atol=1e-14)
    G = O.diff_symbol_sq(shape)
    lam_LtL = np.fft.fftn((L.T @ L)[:, 0].reshape(shape))  # circulant symbol of L^T L
    assert np.allclose(lam_LtL, G, atol=1e-12)


def test_shrink_is_the_proximal_map():
    """u = argmin thr ||u|| + 1/2 ||u - nu||^2 per voxel (step 5b)."""
    rng = np.random.default_rng(13)
    thr = 0.3
    nu = rng.standard_normal((3, 200)) * rng.uniform(0, 1, 200)[None]
    nu[:, 0] = 0.0
    u = O.shrink(nu, thr)
    assert np.all(u[:, 0] == 0.0)
    small = np.sqrt((nu ** 2).sum(0)) <= thr
    assert np.all(u[:, small] == 0.0)

    def f(v, j):
        return thr * np.linalg.norm(v) + 0.5 * np.sum((v - nu[:, j]) ** 2)

    for j in range(nu.shape[1]):
        f0 = f(u[:, j], j)
        for _ in range(10):
            assert f(u[:, j] + 1e-4 * rng.standard_normal(3), j) >= f0 - 1e-15


def _toy_problem(shape=(8, 8, 8), rate=(2, 2, 2), sigma=1.0, seed=20):
    from paper_2010_15491_amd import phantom
    p = phantom.make_problem(shape, rate, sigma, 0.02, seed, n_ellipsoids=4)
    y = O.degrade(p["x_true"], p["psf"], rate) + p["noise"]
    return y, p["psf"], rate


def test_admm_invariants_and_he_yuan_monotonicity():
    """||d_j|| <= lam/mu, d_j parallel to u_j where u_j != 0, and the He-Yuan
    quantity mu||u^{k+1}-u^k||^2 + mu||d^{k+1}-d^k||^2 never increases."""
    y, psf, rate = _toy_problem()
    lam, mu = 0.02, 0.1
    thr = lam / mu
    hy = []

    def cb(it, x, u, d, u1, d1):
        nd = np.sqrt((d1 ** 2).sum(0))
        nu_ = np.sqrt((u1 ** 2).sum(0))
        assert nd.max() <= thr * (1 + 1e-12)
        on = nu_ > 0
        assert np.allclose(d1[:, on], thr * u1[:, on] / nu_[on], atol=1e-12)
        hy.append(mu * np.sum((u1 - u) ** 2) + mu * np.sum((d1 - d) ** 2))

    O.admm_tv(y, psf, rate, lam, mu, 80, callback=cb)
    hy = np.array(hy)
    assert np.all(np.diff(hy) <= 1e-12 * hy[0])


def test_admm_kkt_dual_identity_every_iteration():
    """After step 5a: H^T D^T (DHx - y) + mu L^T d' = -mu L^T (u' - u), exactly.

    Checked with ndimage circular convolution/correlation, at 16^3 with an
    anisotropic rate.
    """
    from paper_2010_15491_amd import phantom
    shape, rate = (16, 16, 16), (2, 2, 4)
    p = phantom.make_problem(shape, rate, 1.2, 0.02, 21, n_ellipsoids=6)
    y = O.degrade(p["x_true"], p["psf"], rate) + p["noise"]
    lam, mu = 2e-3, 5e-2
    psf = p["psf"]

    def cb(it, x, u, d, u1, d1):
        r = O.zero_fill(O.decimate(conv_wrap(x, psf), rate) - y, rate)
        lhs = corr_wrap(r, psf) + mu * O.grad_adjoint(d1)
        rhs = -mu * O.grad_adjoint(u1 - u)
        assert np.abs(lhs - rhs).max() < 1e-11 * max(1.0, np.abs(corr_wrap(
            O.zero_fill(y, rate), psf)).max())

    O.admm_tv(y, psf, rate, lam, mu, 12, callback=cb)


def test_admm_reaches_tv_minimiser_kkt():
    """Run Algorithm 1 long and certify the KKT conditions of the TV problem.

    Stationarity H^T D^T (DHx - y) + lam L^T z = 0 with z = (mu/lam) d,
    ||z_j|| <= 1 and z_j = u_j/||u_j|| where u_j != 0, plus Lx = u. Together
    these make x a minimiser of eq. (3) with isotropic TV. ADMM converges
    sublinearly, so the conditions are checked to the accuracy 3000 iterations
    reach at 8^3, and no nearby point may have a lower objective.
    """
    y, psf, rate = _toy_problem(seed=22)
    lam, mu = 2e-3, 0.2
    res = O.admm_tv(y, psf, rate, lam, mu, 3000, record=True)
    assert res.history[-1][0] < 1e-5 and res.history[-1][1] < 1e-6
    x, u, d = res.x, res.u, res.d
    z = (mu / lam) * d
    r = O.zero_fill(O.decimate(conv_wrap(x, psf), rate) - y, rate)
    stat = corr_wrap(r, psf) + lam * O.grad_adjoint(z)
    scale = np.abs(corr_wrap(O.zero_fill(y, rate), psf)).max()
    assert np.abs(stat).max() < 1e-6 * scale
    assert np.abs(O.grad(x) - u).max() < 1e-5 * np.abs(u).max()
    nz = np.sqrt((z ** 2).sum(0))
    assert nz.max() <= 1 + 1e-9
    nu_ = np.sqrt((u ** 2).sum(0))
    on = nu_ > 1e-6
    assert np.allclose(z[:, on], u[:, on] / nu_[on], atol=1e-6)
    assert np.ptp(x) > 0.1  # a non-trivial (non-constant) minimiser
    f0 = O.tv_objective(x, y, psf, rate, lam)
    rng = np.random.default_rng(0)
    for _ in range(8):
        assert O.tv_objective(x + 1e-2 * rng.standard_normal(x.shape), y, psf, rate, lam) >= f0


def test_aniso_shrink_is_the_componentwise_proximal_map():
    """u = argmin thr ||u||_1 + 1/2 ||u - nu||^2, component by component: the
    minimiser of the scalar problem found by brute force on a fine grid."""
    rng = np.random.default_rng(15)
    thr = 0.3
    nu = rng.standard_normal((3, 60)) * rng.uniform(0, 1.5, 60)[None]
    nu[:, 0] = 0.0
    nu[:, 1] = [thr, -thr, 0.5 * thr]
    u = O.shrink_aniso(nu, thr)
    assert np.all(u[np.abs(nu) <= thr] == 0.0)
    grid = np.linspace(-3.0, 3.0, 600001)
    for v, w in zip(nu.ravel(), u.ravel()):
        f = thr * np.abs(grid) + 0.5 * (grid - v) ** 2
        assert abs(grid[np.argmin(f)] - w) <= 1e-5
    # differs from the isotropic map whenever two components are non-zero
    assert np.abs(u[:, 2:] - O.shrink(nu, thr)[:, 2:]).max() > 1e-2


def test_aniso_equals_iso_when_only_one_axis_varies():
    """With no decimation along n and s the problem is invariant under shifts
    along them, so data constant along n and s keep every iterate constant
    along them: only the m-component of L x is non-zero and both shrinks agree."""
    rng = np.random.default_rng(16)
    shape, rate = (8, 8, 16), (2, 1, 1)
    y1 = rng.standard_normal(shape[2] // rate[0])
    y = np.broadcast_to(y1, O.lr_shape_of(shape, rate)).copy()
    psf = rand_psf(rng, (3, 3, 3))
    a = O.admm_tv(y, psf, rate, 0.02, 0.1, 25)
    b = O.admm_tv(y, psf, rate, 0.02, 0.1, 25, aniso=True)
    assert np.abs(a.x - b.x).max() < 1e-12 * np.abs(a.x).max()
    assert np.abs(O.grad(a.x)[1:]).max() < 1e-12 * np.abs(a.x).max()
    assert np.isclose(O.tv_objective(a.x, y, psf, rate, 0.02),
                      O.tv_objective(a.x, y, psf, rate, 0.02, aniso=True), rtol=1e-12)


def test_aniso_admm_reaches_minimiser_kkt():
    """KKT conditions of the anisotropic TV problem after 3000 iterations at
    8^3: H^T D^T (DHx - y) + lam L^T z = 0 with z = (mu/lam) d, |z_a| <= 1 per
    component and z_a = sign(u_a) where u_a != 0, Lx = u; no nearby point has
    a lower anisotropic objective, and the minimiser is not the isotropic one."""
    y, psf, rate = _toy_problem(seed=25)
    lam, mu = 1e-3, 0.2
    res = O.admm_tv(y, psf, rate, lam, mu, 3000, record=True, aniso=True)
    assert res.history[-1][0] < 1e-5 and res.history[-1][1] < 1e-6
    x, u, d = res.x, res.u, res.d
    z = (mu / lam) * d
    r = O.zero_fill(O.decimate(conv_wrap(x, psf), rate) - y, rate)
    stat = corr_wrap(r, psf) + lam * O.grad_adjoint(z)
    scale = np.abs(corr_wrap(O.zero_fill(y, rate), psf)).max()
    assert np.abs(stat).max() < 1e-6 * scale
    assert np.abs(O.grad(x) - u).max() < 1e-5 * np.abs(u).max()
    assert np.abs(z).max() <= 1 + 1e-9
    on = np.abs(u) > 1e-6
    assert np.allclose(z[on], np.sign(u[on]), atol=1e-6)
    assert np.ptp(x) > 0.1
    f0 = O.tv_objective(x, y, psf, rate, lam, aniso=True)
    rng = np.random.default_rng(1)
    for _ in range(8):
        assert O.tv_objective(x + 1e-2 * rng.standard_normal(x.shape), y, psf, rate, lam,
                              aniso=True) >= f0
    iso = O.admm_tv(y, psf, rate, lam, mu, 3000)
    assert O.rel_l2(iso.x, x) > 1e-4


# ---------------------------------------------------------------------------
# l1 in an orthonormal wavelet basis (3D Haar) through the same x-step
# ---------------------------------------------------------------------------


def _dense_haar(shape, levels):
    n = int(np.prod(shape))
    return np.stack([O.haar3(e.reshape(shape), levels).ravel() for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("shape,levels", [((4, 4, 8), 1), ((4, 8, 4), 2), ((8, 8, 8), 3)])
def test_haar3_is_orthonormal(shape, levels):
    W = _dense_haar(shape, levels)
    assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-13
    c = np.random.default_rng(17).standard_normal(shape)
    assert np.abs(O.haar3_inverse(c, levels).ravel() - W.T @ c.ravel()).max() < 1e-13


def test_haar3_closed_forms():
    """A constant volume has only approximation coefficients, c 2^(3J/2); the
    signal (-1)^m has one non-zero coefficient per 2x2x2 block at level 1,
    sqrt 8 at the block offset (0, 0, 1); a unit impulse at a block's origin
    gives +1/sqrt 8 at all 8 offsets of that block, one at its far corner
    (1, 1, 1) gives (-1)^(a+b+c)/sqrt 8 at offset (a, b, c)."""
    shape = (8, 8, 8)
    for levels in (1, 2, 3):
        c = O.haar3(np.full(shape, 1.5), levels)
        mask = O.haar_detail_mask(shape, levels)
        assert np.abs(c[mask]).max() < 1e-13
        assert np.allclose(c[~mask], 1.5 * 2 ** (1.5 * levels), atol=1e-13)
    alt = np.broadcast_to((-1.0) ** np.arange(8), shape)
    c = O.haar3(alt, 1)
    assert np.allclose(c[0::2, 0::2, 1::2], np.sqrt(8.0), atol=1e-13)
    c[0::2, 0::2, 1::2] = 0.0
    assert np.abs(c).max() < 1e-13
    imp = np.zeros(shape)
    imp[2, 4, 6] = 1.0
    c = O.haar3(imp, 1)
    assert np.allclose(c[2:4, 4:6, 6:8], 1 / np.sqrt(8.0), atol=1e-15)
    c[2:4, 4:6, 6:8] = 0.0
    assert np.abs(c).max() == 0.0
    imp = np.zeros(shape)
    imp[3, 5, 7] = 1.0
    c = O.haar3(imp, 1)
    a_, b_, c_ = np.meshgrid(np.arange(2), np.arange(2), np.arange(2), indexing="ij")
    assert np.allclose(c[2:4, 4:6, 6:8], (-1.0) ** (a_ + b_ + c_) / np.sqrt(8.0), atol=1e-15)


def test_shrink_detail_is_the_proximal_map():
    rng = np.random.default_rng(18)
    thr = 0.25
    nu = rng.standard_normal((4, 4, 4))
    mask = O.haar_detail_mask(nu.shape, 1)
    u = O.shrink_detail(nu, thr, mask)
    assert np.array_equal(u[~mask], nu[~mask])
    grid = np.linspace(-4.0, 4.0, 800001)
    for v, w in zip(nu[mask], u[mask]):
        assert abs(grid[np.argmin(thr * np.abs(grid) + 0.5 * (grid - v) ** 2)] - w) <= 1e-5


def test_wavelet_x_step_solves_the_normal_equations():
    """Step 5a with W: (H^T D^T D H + mu I) x = H^T D^T y + mu W^T (u - d)."""
    rng = np.random.default_rng(19)
    shape, rate, levels = (4, 4, 8), (2, 2, 2), 2
    psf = rand_psf(rng, (3, 3, 3))
    mu = 0.07
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    z = rng.standard_normal(shape)
    H, D, W = dense_H(psf, shape), dense_D(shape, rate), _dense_haar(shape, levels)
    A = H.T @ D.T @ D @ H + mu * np.eye(H.shape[0])
    b = H.T @ D.T @ y.ravel() + mu * W.T @ z.ravel()
    x_dense = np.linalg.solve(A, b).reshape(shape)
    x = O.tikhonov(y, psf, rate, 0.5 * mu, xbar=O.haar3_inverse(z, levels))
    assert np.abs(x - x_dense).max() < 1e-10 * np.abs(x_dense).max()


@pytest.mark.parametrize("levels", [1, 2])
def test_admm_wavelet_reaches_minimiser_kkt(levels):
    """H^T D^T (DHx - y) + lam W^T z = 0 with z = (mu/lam) d, z = 0 on the
    approximation coefficients, |z| <= 1 on the details and z = sign(u) where
    u != 0; W x = u. No nearby point has a lower objective, and the
    regulariser matters (the minimiser differs from the plain least squares
    iterate of the same x-step with d = u = 0). Deblurring without decimation:
    with 2x2x2 decimation the level-1 details are almost invisible to the data
    and every one of them is thresholded to zero."""
    y, psf, rate = _toy_problem(rate=(1, 1, 1), seed=26)
    lam, mu = 2e-3, 0.1
    res = O.admm_wavelet(y, psf, rate, lam, mu, 2000, levels=levels, record=True)
    assert res.history[-1][0] < 1e-6 and res.history[-1][1] < 1e-5
    x, u, d = res.x, res.u, res.d
    mask = O.haar_detail_mask(x.shape, levels)
    z = (mu / lam) * d
    r = O.zero_fill(O.decimate(conv_wrap(x, psf), rate) - y, rate)
    stat = corr_wrap(r, psf) + lam * O.haar3_inverse(z, levels)
    scale = np.abs(corr_wrap(O.zero_fill(y, rate), psf)).max()
    assert np.abs(stat).max() < 1e-6 * scale
    assert np.abs(O.haar3(x, levels) - u).max() < 1e-6 * np.abs(u).max()
    assert np.abs(z[~mask]).max() < 1e-12
    assert np.abs(z[mask]).max() <= 1 + 1e-9
    on = mask & (np.abs(u) > 1e-6)
    assert on.sum() > 0 and np.allclose(z[on], np.sign(u[on]), atol=1e-6)
    assert np.sum(mask & (np.abs(u) == 0)) > 0  # some details are exactly zero
    f0 = O.wavelet_objective(x, y, psf, rate, lam, levels)
    rng = np.random.default_rng(2)
    for _ in range(8):
        assert O.wavelet_objective(x + 1e-2 * rng.standard_normal(x.shape), y, psf, rate, lam,
                                   levels) >= f0
    plain = O.tikhonov(y, psf, rate, 0.5 * mu)
    assert O.rel_l2(plain, x) > 1e-3


def test_admm_large_lambda_gives_constant():
    """lam above the TV kink: the minimiser is the constant mean(y)/Lambda(0)."""
    y, psf, rate = _toy_problem(seed=23)
    res = O.admm_tv(y, psf, rate, 50.0, 1.0, 3000, tol=1e-11)
    c = y.mean() / O.psf_to_otf(psf, O.hr_shape_of(y.shape, rate))[0, 0, 0].real
    assert np.abs(res.x - c).max() < 1e-7


def test_data_term_lr_parseval():
    """1/2||y - DHx||^2 = 1/(2 N_l) || Y - (1/d) fold(Lambda X) ||^2."""
    rng = np.random.default_rng(14)
    shape, rate = (8, 12, 16), (2, 3, 4)
    psf = rand_psf(rng, (3, 3, 3))
    x = rng.standard_normal(shape)
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    otf = O.psf_to_otf(psf, shape)
    d = int(np.prod(rate))
    R = np.fft.fftn(y) - O.fold(otf * np.fft.fftn(x), rate) / d
    assert np.isclose(O.data_term(x, y, otf, rate), 0.5 * np.sum(np.abs(R) ** 2) / y.size,
                      rtol=1e-12)


def test_admm_fixed_count_is_deterministic_and_stops():
    y, psf, rate = _toy_problem(seed=24)
    a = O.admm_tv(y, psf, rate, 0.02, 0.1, 7)
    b = O.admm_tv(y, psf, rate, 0.02, 0.1, 7)
    assert a.iters == 7 and not a.converged
    assert np.array_equal(a.x, b.x)


def test_min_norm_dual_solves_stationarity_with_least_norm():
    """Dense check at 8x8x8: d = pinv(mu L^T) (H^T D^T (y - D H x0)) projected."""
    rng = np.random.default_rng(30)
    shape, rate = (4, 6, 8), (2, 3, 2)
    psf = rand_psf(rng, (3, 3, 3))
    mu = 0.07
    x0 = rng.standard_normal(shape)
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    H, D, L = dense_H(psf, shape), dense_D(shape, rate), dense_L(shape)
    r = H.T @ D.T @ (y.ravel() - D @ H @ x0.ravel())
    d_ref = np.linalg.pinv(mu * L.T) @ r
    d = O.min_norm_dual(x0, y, psf, rate, mu).reshape(-1)
    assert np.allclose(d, d_ref, atol=1e-10)


# ---------------------------------------------------------------------------
# Stopping rule. Algorithm 1 names a stopping criterion without defining it;
# the reading is the relative primal/dual residuals of the ADMM reference the
# paper cites. Pinned with explicit matrices K (= L or the Haar W) on random
# inputs, where either term of max(||Kx||, ||u'||) can be the larger, and on
# the recorded history of real runs, with (u', d') recomputed from steps 5b/5c.
# ---------------------------------------------------------------------------


def _dense_residuals(K, kx, u, u1, d1, mu):
    """Relative residuals from flattened vectors and an explicit matrix K."""
    r = np.linalg.norm(kx - u1)
    s = mu * np.linalg.norm(K.T @ (u1 - u))
    pden = max(np.linalg.norm(kx), np.linalg.norm(u1))
    dden = mu * np.linalg.norm(K.T @ d1)
    return r / pden, s / dden


@pytest.mark.parametrize("u_scale", [0.3, 3.0])
def test_stopping_residuals_match_dense_operators(u_scale):
    """u_scale 3 makes ||u'|| the larger denominator term, 0.3 ||Kx||."""
    rng = np.random.default_rng(40)
    shape, mu = (4, 5, 6), 0.07
    L = dense_L(shape)
    kx, u, u1, d1 = (rng.standard_normal((3,) + shape) for _ in range(4))
    u1 = u_scale * u1
    assert (np.linalg.norm(u1) > np.linalg.norm(kx)) == (u_scale > 1)
    got = O.stopping_residuals(kx, u, u1, d1, O.grad_adjoint, mu)
    ref = _dense_residuals(L, kx.ravel(), u.ravel(), u1.ravel(), d1.ravel(), mu)
    assert np.allclose(got, ref, rtol=1e-12)
    levels, wshape = 2, (4, 4, 8)
    W = _dense_haar(wshape, levels)
    kx, u, u1, d1 = (rng.standard_normal(wshape) for _ in range(4))
    u1 = u_scale * u1
    got = O.stopping_residuals(kx, u, u1, d1, lambda z: O.haar3_inverse(z, levels), mu)
    ref = _dense_residuals(W, kx.ravel(), u.ravel(), u1.ravel(), d1.ravel(), mu)
    assert np.allclose(got, ref, rtol=1e-12)


def _check_history(res, recs):
    assert len(res.history) == len(recs) == res.iters
    h = np.array(res.history)
    # primal = 1 exactly when u' = 0: a trivial run would pin nothing
    assert np.all(np.isfinite(h) & (h > 0)) and np.all(h[:, 0] < 1)
    assert np.allclose(np.array(res.history), np.array(recs), rtol=1e-9, atol=0)


@pytest.mark.parametrize("aniso,warm", [(False, False), (True, False), (False, True)])
def test_admm_tv_history_is_the_dense_stopping_rule(aniso, warm):
    """Every recorded (primal, dual) pair equals the rule evaluated with the
    dense L on that iteration's x, old (u, d) and new (u', d'); (u', d') are
    steps 5b/5c of nu = Lx + d. Along the way ||u'|| <= ||Lx|| (since
    ||d_j|| <= lam/mu), so the primal denominator is ||Lx||."""
    shape = (8, 8, 8)
    y, psf, rate = _toy_problem(seed=27)
    lam, mu = 2e-3, 0.05
    L = dense_L(shape)
    x0 = O.tikhonov(y, psf, rate, 1e-2) if warm else None
    recs = []

    def cb(it, x, u, d, u1, d1):
        lx = L @ x.ravel()
        nu = (lx + d.ravel()).reshape((3,) + shape)
        prox = O.shrink_aniso(nu, lam / mu) if aniso else O.shrink(nu, lam / mu)
        assert np.allclose(u1, prox, rtol=0, atol=1e-13)
        assert np.allclose(d1, nu - prox, rtol=0, atol=1e-13)
        assert np.linalg.norm(u1) <= np.linalg.norm(lx) * (1 + 1e-12)
        recs.append(_dense_residuals(L, lx, u.ravel(), u1.ravel(), d1.ravel(), mu))

    res = O.admm_tv(y, psf, rate, lam, mu, 25, x0=x0, warm_dual=warm, aniso=aniso,
                    record=True, callback=cb)
    _check_history(res, recs)
    assert (res.primal_rel, res.dual_rel) == res.history[-1]


@pytest.mark.parametrize("levels", [1, 2])
def test_admm_wavelet_history_is_the_dense_stopping_rule(levels):
    shape = (4, 4, 8)
    y, psf, rate = _toy_problem(shape=shape, rate=(1, 1, 2), sigma=0.5, seed=28)
    lam, mu = 2e-3, 0.05
    W = _dense_haar(shape, levels)
    mask = O.haar_detail_mask(shape, levels)
    recs = []

    def cb(it, x, u, d, u1, d1):
        wx = W @ x.ravel()
        nu = (wx + d.ravel()).reshape(shape)
        soft = np.sign(nu) * np.maximum(np.abs(nu) - lam / mu, 0.0)
        assert np.allclose(u1, np.where(mask, soft, nu), rtol=0, atol=1e-13)
        assert np.allclose(d1, nu - u1, rtol=0, atol=1e-13)
        recs.append(_dense_residuals(W, wx, u.ravel(), u1.ravel(), d1.ravel(), mu))

    res = O.admm_wavelet(y, psf, rate, lam, mu, 25, levels=levels, record=True, callback=cb)
    _check_history(res, recs)


@pytest.mark.parametrize("tol,tol_dual", [(2e-2, None), (1e-3, 5e-2)])
def test_admm_stops_at_first_iteration_meeting_the_rule(tol, tol_dual):
    """The run stops at the first iteration whose recorded residuals meet the
    tolerances, and not before; a tol = 0 run of the same length records the
    same history."""
    y, psf, rate = _toy_problem(seed=29)
    lam, mu = 2e-3, 0.05
    full = O.admm_tv(y, psf, rate, lam, mu, 400, record=True)
    td = tol_dual or tol
    hits = [i for i, (p, q) in enumerate(full.history) if p <= tol and q <= td]
    assert hits, "tolerance never met; pick a looser one"
    res = O.admm_tv(y, psf, rate, lam, mu, 400, tol=tol, tol_dual=tol_dual, record=True)
    assert res.converged and res.iters == hits[0] + 1
    assert res.history == full.history[: res.iters]
    short = O.admm_tv(y, psf, rate, lam, mu, hits[0], tol=tol, tol_dual=tol_dual)
    assert not short.converged and short.iters == hits[0]


@pytest.mark.parametrize("levels", [1, 2])
def test_wavelet_objective_matches_dense(levels):
    """1/2||y - DHx||^2 + lam sum |detail rows of W applied to x|, with the
    approximation rows of the dense W found on their own: they are the rows
    with a non-zero sum (every detail row is orthogonal to the constants)."""
    rng = np.random.default_rng(31)
    shape, rate, lam = (4, 4, 8), (2, 2, 2), 0.37
    W = _dense_haar(shape, levels)
    approx = np.abs(W.sum(axis=1)) > 1e-9
    assert approx.sum() == W.shape[0] // 8 ** levels
    psf = rand_psf(rng, (3, 3, 3))
    x = rng.standard_normal(shape)
    y = rng.standard_normal(O.lr_shape_of(shape, rate))
    H, D = dense_H(psf, shape), dense_D(shape, rate)
    ref = 0.5 * np.sum((y.ravel() - D @ H @ x.ravel()) ** 2) \
        + lam * np.sum(np.abs(W[~approx] @ x.ravel()))
    assert np.isclose(O.wavelet_objective(x, y, psf, rate, lam, levels), ref, rtol=1e-12)
