"""FP64 CPU oracle of the learned warm-start network (test infrastructure only).

The paper has no network; the warm start is a small 3D CNN applied to the
Tikhonov solution (eq. (12)) to produce the initial x0 of Algorithm 1:
    x0 = x_in + f(x_in),
    f = conv6 o relu o conv5 o ... o relu o conv1,
with 3x3x3 kernels, circular ("same") padding, 32 hidden channels, bias in
every layer and ReLU after layers 1-5. Loss: mean squared error against the
target (the plain TV-ADMM solution); optimiser: Adam.

Conventions shared with the GPU path (stated, not imported):
  * a volume is a C-order array (s, n, m); channels are the leading axis here;
  * tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets dz, dy, dx in {-1,0,1}
    along (s, n, m), and conv(a)[co, v] = sum_t sum_ci W[t, co, ci] a[ci, v+off_t]
    + b[co] (cross-correlation, periodic);
  * parameter vector: for each layer, W as (27, cout, cin) then b (cout,).
  * bf16=True rounds the input, the weights, every stored hidden
    activation (after ReLU) and every stored hidden-layer gradient (after the
    ReLU mask) to bfloat16 (round to nearest even), as the GPU stores them;
    sums are exact (FP64). The output-layer gradient stays unrounded.
"""

from __future__ import annotations

import numpy as np

__all__ = ["LAYERS", "TAPS", "param_count", "unpack", "bf16_round", "conv3d",
           "conv3d_adjoint", "conv3d_weight_grad", "forward", "loss_and_grad", "adam_step"]

CH = 32
LAYERS = [(1, CH), (CH, CH), (CH, CH), (CH, CH), (CH, CH), (CH, 1)]  # (cin, cout)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_count():
    return sum(27 * co * ci + co for ci, co in LAYERS)


def unpack(params):
    """[(W (27, cout, cin), b (cout,))] per layer."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = params[o:o + 27 * co * ci].reshape(27, co, ci)
        o += 27 * co * ci
        b = params[o:o + co]
        o += co
        out.append((W, b))
    return out


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _shift(a, off):
    """a[..., v + off] with periodic wrap over the last three axes."""
    dz, dy, dx = off
    return np.roll(a, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(a, W, b):
    """out[co, v] = sum_t sum_ci W[t, co, ci] a[ci, v + off_t] + b[co]."""
    out = np.zeros((W.shape[1],) + a.shape[1:])
    for t, off in enumerate(TAPS):
        out += np.tensordot(W[t], _shift(a, off), axes=(1, 0))
    return out + b[:, None, None, None]


def conv3d_adjoint(g, W):
    """Adjoint of conv3d in its input: gin[ci, v] = sum_t sum_co W[t, co, ci] g[co, v - off_t]."""
    out = np.zeros((W.shape[2],) + g.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += _shift(np.tensordot(W[t].T, g, axes=(1, 0)), (-dz, -dy, -dx))
    return out


def conv3d_weight_grad(a, g):
    """gW[t, co, ci] = sum_v g[co, v] a[ci, v + off_t]; gb[co] = sum_v g[co, v]."""
    gW = np.stack([np.tensordot(g, _shift(a, off), axes=([1, 2, 3], [1, 2, 3])) for off in TAPS])
    return gW, g.sum(axis=(1, 2, 3))


def forward(params, x, bf16=False):
    """x0 = x + f(x). Returns (x0, cache of layer inputs) for loss_and_grad."""
    rd = bf16_round if bf16 else (lambda v: v)
    layers = [(rd(W), b) for W, b in unpack(np.asarray(params, np.float64))]
    a = rd(np.asarray(x, np.float64))[None]
    cache = []
    for i, (W, b) in enumerate(layers):
        cache.append(a)
        z = conv3d(a, W, b)
        a = rd(np.maximum(z, 0.0)) if i < len(layers) - 1 else z
    return np.asarray(x, np.float64) + a[0], (cache, layers)


def loss_and_grad(params, x, target, bf16=False):
    """Mean squared error of forward(params, x) against target, and its
    gradient with respect to params (backpropagation through the layers)."""
    y, (cache, layers) = forward(params, x, bf16)
    r = y - target
    nv = r.size
    loss = float(np.sum(r * r) / nv)
    g = (2.0 / nv) * r[None]
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a = cache[i]
        gW, gb = conv3d_weight_grad(a, g)
        grads.append((gW, gb))
        if i > 0:
            g = conv3d_adjoint(g, W) * (a > 0)
            if bf16:
                g = bf16_round(g)
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb.ravel()]
    return loss, np.concatenate(flat)


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected, step counted from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
