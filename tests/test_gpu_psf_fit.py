"""PSF estimation (sr3d_psf_fit) on the GPU against the oracle's
fit_gaussian_psf (scipy trust-region least squares on a spatial separable
blur): noise-free data made with a known PSF, gain and offset are recovered
exactly by both; under noise both reach the same minimiser of the same
objective. Inputs: ellipsoid phantoms with texture as the HR reference."""

import numpy as np
import pytest

import oracle as O
from paper_2010_15491_amd import phantom, sr3d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def reference(shape, seed):
    return f32(phantom.make_problem(shape, (1, 1, 1), 1.0, 0.0, seed, texture=True)["x_true"])


@pytest.mark.parametrize("shape,rate,sigma,radius", [
    ((32, 32, 32), (2, 2, 2), (1.6, 1.2, 0.9), (5, 5, 5)),
    ((16, 32, 48), (2, 2, 4), (0.7, 1.9, 1.3), (4, 6, 4)),
    ((24, 24, 24), (1, 2, 2), (2.4, 0.8, 1.1), (7, 3, 4)),
    ((64, 48, 96), (4, 4, 2), (1.3, 1.7, 0.8), (4, 6, 3)),
])
def test_psf_fit_recovers_known_psf(shape, rate, sigma, radius):
    x = reference(shape, 40)
    y = f32(0.85 * O.decimate(O.separable_blur(x, sigma, radius), rate) + 0.07)
    print(f"psf fit {shape} {rate} sigma {sigma}", flush=True)
    r = sr3d.psf_fit(dev(x), dev(y), rate, radius, sigma0=(1.0, 1.0, 1.0))
    print(f"  -> {r}")
    assert r["converged"]
    # y is float32: the minimiser sits within float rounding of the truth
    assert np.allclose(r["sigma"], sigma, rtol=2e-5), r
    assert abs(r["gain"] - 0.85) < 2e-5 and abs(r["offset"] - 0.07) < 2e-5


def test_psf_fit_with_noise_matches_oracle():
    shape, rate, sigma, radius = (48, 48, 48), (2, 2, 2), (1.5, 1.1, 0.8), (5, 5, 5)
    x = reference(shape, 41)
    rng = np.random.default_rng(42)
    y = 0.9 * O.decimate(O.separable_blur(x, sigma, radius), rate) + 0.02
    y = f32(y + 0.01 * rng.standard_normal(y.shape))
    r = sr3d.psf_fit(dev(x), dev(y), rate, radius, sigma0=(1.0, 1.0, 1.0))
    s, a, b, f = O.fit_gaussian_psf(x, y, rate, (1.0, 1.0, 1.0), radius)
    print(f"gpu {r['sigma']} {r['gain']:.6f} {r['offset']:.6f} {r['objective']:.6e}; "
          f"oracle {s} {a:.6f} {b:.6f} {f:.6e}")
    assert r["converged"]
    assert np.allclose(r["sigma"], s, rtol=1e-4) and abs(r["gain"] - a) < 1e-4
    assert abs(r["offset"] - b) < 1e-4
    # the GPU's objective at its fit, evaluated by the oracle's own model
    th = list(r["sigma"]) + [r["gain"], r["offset"]]
    f_gpu = 0.5 * float(np.sum(O.psf_fit_residual(th, x, y, rate, radius) ** 2))
    assert np.isclose(r["objective"], f_gpu, rtol=1e-4)
    assert f_gpu <= f * (1 + 1e-6)
