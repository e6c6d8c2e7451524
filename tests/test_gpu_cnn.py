"""Warm-start CNN on the GPU (BF16 MFMA) against the FP64 CNN oracle.

Single layers get bfloat16-exact inputs and weights on both sides, so their
FP32 outputs must agree to FP32 accumulation error. The whole network rounds
activations and gradients to bfloat16 between layers on both sides; there a
rounding decision can differ where FP32 and FP64 sums straddle a bfloat16
boundary, so the end-to-end bars are looser and stated per test.
"""

import numpy as np
import pytest

import oracle as O
from oracle import cnn_oracle as C
from paper_2010_15491_amd import phantom, sr3d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def bf(a):
    return C.bf16_round(a)


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def devbf(a_cl):
    """channels-last array (s, n, m, 32) -> CUDA bfloat16 (values must be bf16-exact)."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a_cl, np.float32))).cuda().to(
        torch.bfloat16)


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().double().cpu().numpy()


def cl(a):  # (C, s, n, m) -> (s, n, m, C)
    return np.moveaxis(a, 0, -1)


def cf(a):  # (s, n, m, C) -> (C, s, n, m)
    return np.moveaxis(a, -1, 0)


SHAPES = [(16, 12, 24), (8, 8, 8), (5, 6, 7), (9, 20, 72), (1, 2, 3)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_1_to_32_forward(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape)
    W = bf(rng.standard_normal((27, 32, 1)) * 0.3)
    b = rng.standard_normal(32) * 0.1
    out, out32 = sr3d.conv3d_forward(shape, dev32(W), dev32(b), x=dev32(x))
    ref = np.maximum(C.conv3d(bf(x)[None], W, np.float32(b).astype(np.float64)), 0)
    got = cf(host(out32))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-6
    assert np.array_equal(cf(host(out)), bf(got))


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_32_to_32_forward_mfma(shape):
    rng = np.random.default_rng(2)
    a = bf(rng.standard_normal((32,) + shape))
    W = bf(rng.standard_normal((27, 32, 32)) * 0.05)
    b = np.float32(rng.standard_normal(32) * 0.1).astype(np.float64)
    out, out32 = sr3d.conv3d_forward(shape, dev32(W), dev32(b), act=devbf(cl(a)))
    ref = np.maximum(C.conv3d(a, W, b), 0)
    got = cf(host(out32))
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()
    assert np.array_equal(cf(host(out)), bf(got))


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_32_to_32_backward_mfma(shape):
    rng = np.random.default_rng(3)
    a = bf(np.maximum(rng.standard_normal((32,) + shape), 0))
    g = bf(rng.standard_normal((32,) + shape) * 0.01)
    W = bf(rng.standard_normal((27, 32, 32)) * 0.05)
    gw, gin, gin32 = sr3d.conv3d_backward(shape, devbf(cl(a)), devbf(cl(g)), dev32(W),
                                          mask=devbf(cl(a)))
    gW_ref, gb_ref = C.conv3d_weight_grad(a, g)
    gw = host(gw)
    assert np.abs(gw[:27 * 1024] - gW_ref.ravel()).max() < 1e-5 * np.abs(gW_ref).max()
    assert np.abs(gw[27 * 1024:] - gb_ref).max() < 1e-5 * np.abs(gb_ref).max()
    gin_ref = C.conv3d_adjoint(g, W) * (a > 0)
    got = cf(host(gin32))
    assert np.abs(got - gin_ref).max() < 1e-5 * np.abs(gin_ref).max()
    assert np.array_equal(cf(host(gin)), bf(got))


def test_adam_matches_oracle():
    n = sr3d.cnn_param_count()
    assert n == C.param_count()
    rng = np.random.default_rng(4)
    p, m, v = rng.standard_normal(n), np.zeros(n), np.zeros(n)
    P, Mm, V = dev32(p), dev32(m), dev32(v)
    for step in range(1, 4):
        g = rng.standard_normal(n)
        p, m, v = C.adam_step(p, np.float32(g).astype(np.float64), m, v, step, 1e-3)
        sr3d.cnn_adam(P, dev32(g), Mm, V, step, 1e-3)
    assert np.abs(host(P) - p).max() < 1e-5


def test_init_is_seeded_and_scaled():
    a, b, c = sr3d.cnn_init(7), sr3d.cnn_init(7), sr3d.cnn_init(8)
    assert torch.equal(a, b) and not torch.equal(a, c)
    layers = C.unpack(host(a))
    for (W, bb), (ci, co) in zip(layers, C.LAYERS):
        lim = np.sqrt(6.0 / (27 * ci)) * (0.1 if co == 1 else 1.0)
        assert np.abs(W).max() <= lim and np.abs(W).max() > 0.5 * lim
        assert np.all(bb == 0)


def _net_case(shape, seed):
    rng = np.random.default_rng(seed)
    p = np.float32(rng.standard_normal(C.param_count()) * 0.05).astype(np.float64)
    o = 0
    for ci, co in C.LAYERS:  # keep biases small but nonzero
        o += 27 * co * ci
        p[o:o + co] *= 0.2
        o += co
    x = rng.standard_normal(shape)
    t = x + 0.05 * rng.standard_normal(shape)
    return p, x, t


def test_network_forward_matches_bf16_oracle():
    shape = (16, 16, 24)
    p, x, _ = _net_case(shape, 5)
    y = host(sr3d.cnn_forward(dev32(p), dev32(x)))
    ref, _ = C.forward(p, np.float32(x).astype(np.float64), bf16=True)
    fx, fr = y - np.float32(x), ref - np.float32(x)
    # bfloat16 rounding of hidden activations may differ by one unit where the
    # FP32 and FP64 sums straddle a rounding boundary
    assert np.linalg.norm(fx - fr) / np.linalg.norm(fr) < 5e-3


def test_network_gradient_matches_bf16_oracle():
    shape = (12, 16, 16)
    p, x, t = _net_case(shape, 6)
    x32, t32 = np.float32(x).astype(np.float64), np.float32(t).astype(np.float64)
    loss, g = sr3d.cnn_grad(dev32(p), dev32(x32), dev32(t32))
    loss_ref, g_ref = C.loss_and_grad(p, x32, t32, bf16=True)
    assert abs(float(host(loss)[0]) - loss_ref) < 1e-4 * loss_ref
    g = host(g)
    o = 0
    for ci, co in C.LAYERS:
        n = 27 * co * ci + co
        err = np.linalg.norm(g[o:o + n] - g_ref[o:o + n]) / np.linalg.norm(g_ref[o:o + n])
        assert err < 2e-2, (ci, co, err)
        o += n


def test_training_lowers_loss_and_the_warm_start_gains():
    """A few hundred Adam steps on Tikhonov -> TV-ADMM pairs at 32^3: the loss
    drops, and on a held-out volume the network's x0 is closer to the ADMM
    solution than the Tikhonov input it started from."""
    shape, rate, lam, mu = (32, 32, 32), (2, 2, 2), 2e-3, 5e-2
    pairs = []
    for seed in range(1000, 1007):
        pr = phantom.make_problem(shape, rate, 1.5, 0.02, seed, n_ellipsoids=12)
        P = dev32(pr["psf"])
        Y = sr3d.degrade(dev32(pr["x_true"]), P, rate) + dev32(pr["noise"])
        xt = sr3d.tikhonov(Y, P, rate, 1e-3)
        xa, _ = sr3d.tv_admm(Y, P, rate, lam, mu, 200, tol=1e-4)
        pairs.append((xt, xa))
    train, held = pairs[:-1], pairs[-1]
    params = sr3d.cnn_init(11)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    ws = sr3d.CnnWorkspace(shape)
    first = last = None
    for step in range(1, 301):
        xt, xa = train[step % len(train)]
        loss, g = sr3d.cnn_grad(params, xt, xa, ws=ws)
        sr3d.cnn_adam(params, g, m, v, step, 1e-3)
        lv = float(loss.item())
        first = lv if first is None else first
        last = lv
    assert last < 0.5 * first, (first, last)
    xt, xa = held
    x0 = sr3d.cnn_forward(params, xt, ws=ws)
    e_tik = float(torch.linalg.vector_norm(xt - xa))
    e_cnn = float(torch.linalg.vector_norm(x0 - xa))
    print(f"held-out distance to the ADMM solution: Tikhonov {e_tik:.4f}, CNN {e_cnn:.4f}")
    assert e_cnn < 0.8 * e_tik


def test_warm_solve_accepts_or_falls_back_to_plain_admm():
    """warmstart.solve: the learned start is kept only when its ADMM run meets
    the tolerance; otherwise plain ADMM (x0 = 0) runs and its x is returned,
    bit-equal to a plain solve with the same tolerance and cap."""
    from paper_2010_15491_amd import warmstart
    shape, rate, lam, mu = (32, 32, 32), (2, 2, 2), 2e-3, 5e-2
    pr = phantom.make_problem(shape, rate, 1.5, 0.02, 1010)
    P = dev32(pr["psf"])
    Y = sr3d.degrade(dev32(pr["x_true"]), P, rate) + dev32(pr["noise"])
    params = sr3d.cnn_init(3)
    # accept: a loose tolerance that the warm-started run meets
    x, info = warmstart.solve(params, Y, P, rate, lam, mu, 200, tol=2e-2)
    assert info.used == "warm" and info.warm.converged and info.plain is None
    x0 = warmstart.warm_start(params, Y, P, rate)
    xw, stw = sr3d.tv_admm(Y, P, rate, lam, mu, 200, tol=2e-2, x0=x0)
    assert torch.equal(x, xw) and stw.iters == info.warm.iters
    # fall back: a tolerance no run reaches within 5 iterations
    x, info = warmstart.solve(params, Y, P, rate, lam, mu, 5, tol=1e-9)
    assert info.used == "plain" and not info.warm.converged and info.warm.iters == 5
    xp, stp = sr3d.tv_admm(Y, P, rate, lam, mu, 5, tol=1e-9)
    assert torch.equal(x, xp) and info.plain.iters == stp.iters == 5
