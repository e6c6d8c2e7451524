"""Pins of the oracle's l1 data term (non-Gaussian noise, Sec. V) on the CPU.

The method: min_x ||D H x - y||_1 + lam TV(x) by ADMM with the splits
u = L x and v = D H x - y. The pins use what the oracle does not share:
dense D, H and L built voxel by voxel, a brute-force scalar prox, a linear
program solved by scipy's HiGHS for the anisotropic form (an LP with dense
matrices), and the optimality (KKT) conditions of the isotropic form.
"""

import numpy as np
import pytest
from scipy.optimize import linprog

import oracle as O
from test_oracle_pins import dense_D, dense_H, dense_L, rand_psf


def impulse_problem(shape, rate, seed, frac=0.1, amp=1.5, sigma=0.5):
    """Ellipsoid phantom, Gaussian blur, decimation, then impulse noise on a
    fraction of the LR voxels (the noise an l1 data term is for)."""
    from paper_2010_15491_amd import phantom
    p = phantom.make_problem(shape, rate, sigma, 0.0, seed, n_ellipsoids=4)
    y = O.degrade(p["x_true"], p["psf"], rate)
    rng = np.random.default_rng(seed + 1)
    hit = rng.random(y.shape) < frac
    y = y + hit * rng.choice([-amp, amp], size=y.shape)
    return y, p["psf"], p["x_true"]


def test_soft_is_the_proximal_map():
    """soft(z, t) = argmin_v t|v| + 1/2 (v - z)^2, by brute force on a grid."""
    grid = np.linspace(-4, 4, 80001)
    for z in (-2.3, -0.4, 0.0, 0.25, 1.7):
        for t in (0.1, 0.5, 2.0):
            f = t * np.abs(grid) + 0.5 * (grid - z) ** 2
            assert abs(O.soft(np.array(z), t) - grid[np.argmin(f)]) <= 1e-4


def _dense_ops(shape, rate, psf):
    H = dense_H(psf, shape)
    D = dense_D(shape, rate)
    return D @ H, dense_L(shape)


def test_l1data_x_step_stationarity_every_iteration():
    """After every x-update, with dense operators:
    mu_data (DH)^T (DHx - y - v + e) + mu L^T (Lx - u + d) = 0."""
    shape, rate = (4, 8, 8), (2, 2, 1)
    y, psf, _ = impulse_problem(shape, rate, 70)
    lam, mu, mu_d = 5e-3, 0.05, 2.0
    A, L = _dense_ops(shape, rate, psf)

    def cb(it, x, u, d, u1, d1, v, e, v1, e1):
        xv = x.ravel()
        g = (mu_d * A.T @ (A @ xv - y.ravel() - v.ravel() + e.ravel())
             + mu * L.T @ (L @ xv - u.ravel() + d.ravel()))
        assert np.abs(g).max() < 1e-11 * max(1.0, mu_d * np.abs(A.T @ y.ravel()).max())

    O.admm_l1data(y, psf, rate, lam, mu, mu_d, 15, callback=cb)


@pytest.mark.parametrize("aniso", [False, True])
def test_l1data_history_is_the_dense_stopping_rule(aniso):
    """Steps 5b/5c and 5b'/5c' recomputed with dense matrices, and every
    recorded residual equal to the rule evaluated with them: both splits'
    primal and dual, and the reported max of each kind."""
    shape, rate = (4, 8, 8), (2, 2, 1)
    y, psf, _ = impulse_problem(shape, rate, 71)
    lam, mu, mu_d = 5e-2, 0.05, 2.0
    A, L = _dense_ops(shape, rate, psf)
    yv = y.ravel()
    recs = []

    def cb(it, x, u, d, u1, d1, v, e, v1, e1):
        xv = x.ravel()
        lx, t = L @ xv, A @ xv
        nu = lx + d.ravel()
        if aniso:
            pu = np.sign(nu) * np.maximum(np.abs(nu) - lam / mu, 0.0)
        else:
            nn = np.sqrt((nu.reshape(3, -1) ** 2).sum(0))
            sc = np.where(nn > 0, np.maximum(nn - lam / mu, 0.0) / np.where(nn > 0, nn, 1), 0.0)
            pu = (nu.reshape(3, -1) * sc).ravel()
        assert np.allclose(u1.ravel(), pu, rtol=0, atol=1e-13)
        assert np.allclose(d1.ravel(), nu - pu, rtol=0, atol=1e-13)
        a = t - yv + e.ravel()
        pv = np.sign(a) * np.maximum(np.abs(a) - 1.0 / mu_d, 0.0)
        assert np.allclose(v1.ravel(), pv, rtol=0, atol=1e-13)
        assert np.allclose(e1.ravel(), a - pv, rtol=0, atol=1e-13)
        p_tv = np.linalg.norm(lx - u1.ravel()) / max(np.linalg.norm(lx), np.linalg.norm(u1))
        d_tv = np.linalg.norm(L.T @ (u1 - u).ravel()) / np.linalg.norm(L.T @ d1.ravel())
        p_da = (np.linalg.norm(t - v1.ravel() - yv)
                / max(np.linalg.norm(t), np.linalg.norm(v1), np.linalg.norm(yv)))
        d_da = np.linalg.norm(A.T @ (v1 - v).ravel()) / np.linalg.norm(A.T @ e1.ravel())
        recs.append((max(p_tv, p_da), max(d_tv, d_da), p_tv, d_tv, p_da, d_da))

    res = O.admm_l1data(y, psf, rate, lam, mu, mu_d, 20, aniso=aniso, record=True, callback=cb)
    h = np.array(res.history)
    assert h.shape == (20, 6) and np.all(np.isfinite(h)) and np.all(h[:, :5] > 0)
    if not aniso:
        # each split decides the reported primal and the reported dual
        # somewhere along this run (a rule reporting one split only fails)
        assert np.any(h[:, 2] > h[:, 4]) and np.any(h[:, 4] > h[:, 2])
        assert np.any(h[:, 3] > h[:, 5]) and np.any(h[:, 5] > h[:, 3])
    assert np.allclose(h, np.array(recs), rtol=1e-9, atol=0)
    assert (res.primal_rel, res.dual_rel) == tuple(res.history[-1][:2])


def test_l1data_aniso_reaches_the_linear_program_optimum():
    """With anisotropic TV the problem min ||DHx - y||_1 + lam ||Lx||_1 is a
    linear program: min 1's + lam 1't s.t. -s <= DHx - y <= s, -t <= Lx <= t.
    HiGHS solves it exactly; ADMM run long must reach the same optimal value
    (the minimiser of an LP need not be unique, its value is)."""
    shape, rate = (4, 4, 8), (2, 2, 1)
    y, psf, _ = impulse_problem(shape, rate, 72)
    psf = rand_psf(np.random.default_rng(3), (3, 3, 3))
    lam = 0.02
    A, L = _dense_ops(shape, rate, psf)
    n, m, k = A.shape[1], A.shape[0], L.shape[0]
    c = np.concatenate([np.zeros(n), np.ones(m), lam * np.ones(k)])
    I_m, I_k = np.eye(m), np.eye(k)
    Aub = np.block([[A, -I_m, np.zeros((m, k))], [-A, -I_m, np.zeros((m, k))],
                    [L, np.zeros((k, m)), -I_k], [-L, np.zeros((k, m)), -I_k]])
    bub = np.concatenate([y.ravel(), -y.ravel(), np.zeros(k), np.zeros(k)])
    bounds = [(None, None)] * n + [(0, None)] * (m + k)
    lp = linprog(c, A_ub=Aub, b_ub=bub, bounds=bounds, method="highs")
    assert lp.status == 0
    res = O.admm_l1data(y, psf, rate, lam, 0.05, 1.0, 6000, aniso=True)
    f = O.l1data_objective(res.x, y, psf, rate, lam, aniso=True)
    f_lp = O.l1data_objective(lp.x[:n].reshape(shape), y, psf, rate, lam, aniso=True)
    assert abs(f_lp - lp.fun) < 1e-9 * lp.fun  # the objective as the LP states it
    assert f >= lp.fun * (1 - 1e-9)
    assert f - lp.fun < 1e-5 * lp.fun, (f, lp.fun)


def test_l1data_reaches_minimiser_kkt():
    """Isotropic form, run long: with p = mu_data e and q = mu d the
    optimality conditions are (DH)^T p + L^T q = 0, |p_i| <= 1 with
    p_i = sign(DHx - y)_i where DHx - y != 0, ||q_j|| <= lam with
    q_j = lam (Lx)_j / ||(Lx)_j|| where (Lx)_j != 0, checked with dense
    matrices to the accuracy 4000 iterations reach (ADMM converges
    sublinearly); no nearby point may have a lower objective."""
    shape, rate = (4, 8, 8), (2, 2, 1)
    y, psf, _ = impulse_problem(shape, rate, 73)
    lam, mu, mu_d = 0.08, 0.3, 5.0
    res = O.admm_l1data(y, psf, rate, lam, mu, mu_d, 4000, record=True)
    assert res.history[-1][0] < 1e-4 and res.history[-1][1] < 1e-5
    A, L = _dense_ops(shape, rate, psf)
    x = res.x.ravel()
    p, q = mu_d * res.e.ravel(), mu * res.d.ravel()
    stat = A.T @ p + L.T @ q
    assert np.abs(stat).max() < 1e-4
    r = A @ x - y.ravel()
    assert np.abs(p).max() <= 1 + 1e-9
    big = np.abs(r) > 1e-3
    assert big.sum() >= 3 and np.allclose(p[big], np.sign(r[big]), atol=1e-3)
    lx = (L @ x).reshape(3, -1)
    qv = q.reshape(3, -1)
    assert np.sqrt((qv ** 2).sum(0)).max() <= lam * (1 + 1e-9)
    nl = np.sqrt((lx ** 2).sum(0))
    on = nl > 0.05  # edges resolved well beyond the run's residuals
    assert on.sum() > 10 and np.allclose(qv[:, on], lam * lx[:, on] / nl[on], atol=1e-3 * lam)
    assert np.ptp(res.x) > 0.5  # a non-trivial minimiser
    f0 = O.l1data_objective(res.x, y, psf, rate, lam)
    rng = np.random.default_rng(1)
    for _ in range(8):
        assert O.l1data_objective(res.x + 1e-3 * rng.standard_normal(res.x.shape), y, psf,
                                  rate, lam) >= f0


def test_l1data_removes_impulses_that_l2_keeps():
    """Why the l1 data term is there: with impulse noise on 10% of the LR
    voxels, the l1 solution is closer to the clean volume than the l2 one
    (Algorithm 1) at the same lam."""
    shape, rate = (16, 16, 16), (2, 2, 2)
    y, psf, xt = impulse_problem(shape, rate, 74, frac=0.1, amp=2.0, sigma=1.0)
    lam = 0.03
    x1 = O.admm_l1data(y, psf, rate, lam, 0.05, 1.0, 300).x
    x2 = O.admm_tv(y, psf, rate, lam, 0.05, 300).x
    assert O.rel_l2(x1, xt) < 0.5 * O.rel_l2(x2, xt)
