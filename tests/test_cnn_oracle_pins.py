"""Pins of the FP64 warm-start CNN oracle (CPU only): scipy.ndimage's periodic
correlation, adjoint (dot-product) identities, central finite differences of
the loss, torch's bfloat16 rounding and torch's Adam."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn_oracle as C


def rand_params(rng, scale=0.2):
    return rng.standard_normal(C.param_count()) * scale


def test_conv3d_matches_ndimage_correlate():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3, 5, 6, 7))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    out = C.conv3d(a, W, b)
    for co in range(2):
        ref = np.full(a.shape[1:], b[co])
        for ci in range(3):
            k = W[:, co, ci].reshape(3, 3, 3)  # k[dz+1, dy+1, dx+1]
            ref += ndimage.correlate(a[ci], k, mode="wrap")
        assert np.allclose(out[co], ref, atol=1e-12)


def test_conv3d_adjoint_and_weight_grad_identities():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((4, 4, 5, 6))
    g = rng.standard_normal((3, 4, 5, 6))
    W = rng.standard_normal((27, 3, 4))
    lhs = np.sum(C.conv3d(a, W, np.zeros(3)) * g)
    assert np.isclose(lhs, np.sum(a * C.conv3d_adjoint(g, W)), rtol=1e-12)
    gW, gb = C.conv3d_weight_grad(a, g)
    assert np.isclose(lhs, np.sum(W * gW), rtol=1e-12)
    assert np.allclose(gb, g.sum(axis=(1, 2, 3)))


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    shape = (4, 4, 4)
    x = rng.standard_normal(shape)
    t = x + 0.1 * rng.standard_normal(shape)
    p = rand_params(rng)
    loss, g = C.loss_and_grad(p, x, t)
    idx = rng.choice(p.size, 40, replace=False)
    # every layer's weights and biases represented
    o = 0
    for ci, co in C.LAYERS:
        idx = np.concatenate([idx, [o, o + 27 * co * ci]])
        o += 27 * co * ci + co
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (C.loss_and_grad(p + e, x, t)[0] - C.loss_and_grad(p - e, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(v), ref)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = C.adam_step(p, g, m, v, step, 1e-2)
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(p, tp.detach().numpy(), atol=1e-12)


def test_bf16_forward_is_close_to_exact_forward():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((6, 6, 6))
    p = rand_params(rng, 0.1)
    y64, _ = C.forward(p, x)
    y16, _ = C.forward(p, x, bf16=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 2e-2
