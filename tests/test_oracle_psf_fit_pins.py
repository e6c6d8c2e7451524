"""Pins of the oracle's PSF estimation (Sec. IV-B: a 3D Gaussian fitted to
the data; the paper gives only the fitted widths). Reading: with an HR
reference x and the LR volume y, (sigma, gain, offset) minimise
1/2 ||y - alpha D H_sigma x - beta||^2 over a separable sampled Gaussian on a
fixed support. The pins use the FFT-based forward model of the oracle's
degradation (eq. (1)-(2)), exact recovery from noise-free data, and
first-order optimality checked by finite differences."""

import numpy as np
import pytest

import oracle as O
from paper_2010_15491_amd import phantom


def reference(shape, seed, texture=True):
    return phantom.make_problem(shape, (1, 1, 1), 1.0, 0.0, seed, texture=texture)["x_true"]


@pytest.mark.parametrize("sigma", [(1.0, 1.0, 1.0), (1.7, 1.2, 0.6), (0.8, 2.1, 1.4)])
def test_separable_blur_is_the_degradation_blur(sigma):
    """With radius ceil(2 sigma) per axis the fitted model's kernel is the
    sampled Gaussian PSF of the input recipe, and its spatial separable blur
    equals the Fourier-domain blur of eq. (2)."""
    x = reference((24, 32, 28), 30)
    radius = tuple(int(np.ceil(2 * s - 1e-12)) for s in sigma)
    psf = phantom.gaussian_psf(sigma)
    assert psf.shape == tuple(2 * r + 1 for r in radius[::-1])
    ref = O.blur(x, O.psf_to_otf(psf, x.shape))
    assert np.abs(O.separable_blur(x, sigma, radius) - ref).max() < 1e-12
    taps = O.gaussian_taps(sigma[0], radius[0])
    assert np.isclose(taps.sum(), 1.0) and np.allclose(taps, taps[::-1])


@pytest.mark.parametrize("shape,rate,sigma,radius", [
    ((32, 32, 32), (2, 2, 2), (1.6, 1.2, 0.9), (5, 5, 5)),
    ((16, 32, 48), (2, 2, 4), (0.7, 1.9, 1.3), (4, 6, 4)),
    ((24, 24, 24), (1, 2, 2), (2.4, 0.8, 1.1), (7, 3, 4)),
])
def test_fit_recovers_known_sigma_gain_offset(shape, rate, sigma, radius):
    """Noise-free data made with a known PSF, gain and offset: the fit
    returns them (the least-squares minimum is zero there)."""
    x = reference(shape, 31)
    y = 0.85 * O.decimate(O.separable_blur(x, sigma, radius), rate) + 0.07
    s, a, b, f = O.fit_gaussian_psf(x, y, rate, (1.0, 1.0, 1.0), radius)
    assert np.allclose(s, sigma, rtol=1e-8) and abs(a - 0.85) < 1e-8 and abs(b - 0.07) < 1e-8
    assert f < 1e-20


def test_fit_with_noise_is_a_stationary_minimum_near_the_truth():
    """Gaussian noise on y: the estimate stays close to the truth, its
    residual is no larger than the truth's, and the objective's gradient
    (central differences) vanishes there."""
    shape, rate, sigma, radius = (32, 32, 32), (2, 2, 2), (1.5, 1.1, 0.8), (5, 5, 5)
    x = reference(shape, 32)
    rng = np.random.default_rng(33)
    y = 0.9 * O.decimate(O.separable_blur(x, sigma, radius), rate) + 0.02
    y = y + 0.01 * rng.standard_normal(y.shape)
    s, a, b, f = O.fit_gaussian_psf(x, y, rate, (1.0, 1.0, 1.0), radius)
    assert np.allclose(s, sigma, rtol=3e-2) and abs(a - 0.9) < 3e-2
    th = np.array(list(s) + [a, b])

    def obj(t):
        r = O.psf_fit_residual(t, x, y, rate, radius)
        return 0.5 * float(r @ r)

    assert abs(obj(th) - f) < 1e-12 * f
    assert f <= obj(np.array(list(sigma) + [0.9, 0.02]))
    for i in range(5):
        h = 1e-5 * max(1.0, abs(th[i]))
        e = np.zeros(5)
        e[i] = h
        g = (obj(th + e) - obj(th - e)) / (2 * h)
        assert abs(g) < 1e-6 * f / max(abs(th[i]), 1e-3), (i, g)
