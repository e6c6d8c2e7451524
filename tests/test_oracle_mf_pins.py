"""Pins of the oracle's multi-frame SR (Sec. V, future work): F LR frames
y_f = D S_f H x + n_f with known HR shifts t_f. Pinned by the single-frame
oracle (F = 1, t = 0), dense normal equations built voxel by voxel, the
stationarity of every multi-frame x-update with ndimage operators, explicit
indexing of the shifted decimation, and the exact closed form when the frames
cover every voxel of a block and the PSF is a delta."""

import itertools

import numpy as np
import pytest

import oracle as O
from paper_2010_15491_amd import phantom
from test_oracle_pins import conv_wrap, corr_wrap, dense_D, dense_H, rand_psf


def frames(x, psf, rate, shifts, noise, seed):
    rng = np.random.default_rng(seed)
    hx = conv_wrap(x, psf)
    return [O.decimate(O.shift(hx, t), rate) + noise * rng.standard_normal(
        O.lr_shape_of(x.shape, rate)) for t in shifts]


def dense_S(shape, t):
    """Permutation matrix of (S z)[i] = z[i + t] (circular)."""
    S, N, M = shape
    n = S * N * M
    P = np.zeros((n, n))
    for s in range(S):
        for q in range(N):
            for m in range(M):
                i = (s * N + q) * M + m
                j = (((s + t[2]) % S) * N + (q + t[1]) % N) * M + (m + t[0]) % M
                P[i, j] = 1.0
    return P


def test_shifted_decimation_is_explicit_indexing():
    """y_f[j] = (Hx)[j r + t_f] per axis: the frame samples the blurred volume
    at offset t_f inside every block."""
    S, N, M = 8, 12, 16
    dr, dc, ds = 2, 3, 2
    x = np.random.default_rng(1).standard_normal((S, N, M))
    for t in [(1, 0, 0), (0, 2, 1), (3, 1, 1), (17, 5, 9)]:
        y = O.decimate(O.shift(x, t), (dr, dc, ds))
        ref = np.empty((S // ds, N // dc, M // dr))
        for js in range(S // ds):
            for jn in range(N // dc):
                for jm in range(M // dr):
                    ref[js, jn, jm] = x[(js * ds + t[2]) % S, (jn * dc + t[1]) % N,
                                        (jm * dr + t[0]) % M]
        assert np.array_equal(y, ref)


def test_one_unshifted_frame_is_the_single_frame_method():
    shape, rate = (8, 16, 16), (2, 2, 2)
    p = phantom.make_problem(shape, rate, 0.6, 0.01, 5)
    y = O.degrade(p["x_true"], p["psf"], rate) + p["noise"]
    xbar = np.random.default_rng(2).standard_normal(shape) * 0.1
    a = O.tikhonov_mf([y], [(0, 0, 0)], p["psf"], rate, 1e-2, xbar)
    assert np.abs(a - O.tikhonov(y, p["psf"], rate, 1e-2, xbar)).max() < 1e-12
    r1 = O.admm_tv_mf([y], [(0, 0, 0)], p["psf"], rate, 2e-3, 5e-2, 6)
    r2 = O.admm_tv(y, p["psf"], rate, 2e-3, 5e-2, 6)
    assert np.abs(r1.x - r2.x).max() < 1e-12 and np.isclose(r1.dual_rel, r2.dual_rel, rtol=1e-9)


@pytest.mark.parametrize("shape,rate,shifts", [
    ((8, 8, 8), (2, 2, 2), [(0, 0, 0), (1, 0, 1), (1, 1, 0)]),
    ((4, 8, 12), (2, 2, 1), [(1, 1, 0), (0, 1, 0)]),
    ((8, 4, 8), (4, 2, 2), [(0, 0, 0), (3, 1, 1), (2, 0, 1), (1, 1, 0)]),
])
def test_tikhonov_mf_matches_dense_normal_equations(shape, rate, shifts):
    rng = np.random.default_rng(3)
    psf = rand_psf(rng, (3, 3, 3))
    x = rng.standard_normal(shape)
    ys = frames(x, psf, rate, shifts, 0.05, 4)
    lam, xbar = 3e-2, 0.1 * rng.standard_normal(shape)
    H, D = dense_H(psf, shape), dense_D(shape, rate)
    n = H.shape[0]
    lhs = 2 * lam * np.eye(n)
    rhs = 2 * lam * xbar.ravel()
    for y, t in zip(ys, shifts):
        Af = D @ dense_S(shape, t) @ H
        lhs += Af.T @ Af
        rhs += Af.T @ y.ravel()
    ref = np.linalg.solve(lhs, rhs).reshape(shape)
    got = O.tikhonov_mf(ys, shifts, psf, rate, lam, xbar)
    assert np.abs(got - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_admm_tv_mf_x_update_stationarity_every_iteration():
    """After step 5a: sum_f H^T S_f^T D^T (D S_f H x - y_f) + mu L^T (L x - u + d) = 0,
    with ndimage circular convolution and correlation."""
    shape, rate = (16, 16, 16), (2, 2, 2)
    shifts = [(0, 0, 0), (1, 1, 0), (0, 1, 1)]
    p = phantom.make_problem(shape, rate, 1.0, 0.0, 6, n_ellipsoids=6)
    psf = p["psf"]
    ys = frames(p["x_true"], psf, rate, shifts, 0.02, 7)
    lam, mu = 2e-3, 5e-2

    def cb(it, x, u, d, u1, d1):
        hx = conv_wrap(x, psf)
        g = np.zeros(shape)
        for y, t in zip(ys, shifts):
            r = O.zero_fill(O.decimate(O.shift(hx, t), rate) - y, rate)
            g += corr_wrap(O.shift(r, tuple(-v for v in t)), psf)
        g += mu * O.grad_adjoint(O.grad(x) - u + d)
        scale = np.abs(corr_wrap(O.zero_fill(ys[0], rate), psf)).max()
        assert np.abs(g).max() < 1e-11 * scale

    O.admm_tv_mf(ys, shifts, psf, rate, lam, mu, 8, callback=cb)


def test_frames_covering_every_block_offset_with_delta_psf_give_the_closed_form():
    """All d block offsets observed once each and H = I: every HR voxel is
    seen exactly once, so the Tikhonov minimiser is (y + 2 lam xbar)/(1 + 2 lam)
    with y the interleaved frames."""
    shape, rate = (8, 8, 12), (2, 2, 2)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(shape)
    xbar = rng.standard_normal(shape)
    shifts = list(itertools.product(range(2), range(2), range(2)))
    delta = np.zeros((1, 1, 1))
    delta[0, 0, 0] = 1.0
    ys = [O.decimate(O.shift(x, t), rate) for t in shifts]
    lam = 0.05
    got = O.tikhonov_mf(ys, shifts, delta, rate, lam, xbar)
    assert np.abs(got - (x + 2 * lam * xbar) / (1 + 2 * lam)).max() < 1e-12
