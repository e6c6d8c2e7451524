"""The l1 data term (SR3D_DATA_L1, non-Gaussian noise) on the GPU against the
FP64 oracle's admm_l1data, through the C ABI. Inputs: ellipsoid phantoms,
Gaussian blur and decimation by the oracle, Gaussian noise plus impulses on
10% of the LR voxels; both sides get the same float32-rounded y, PSF and x0.
Bar: rel-L2 <= 1e-5 and max |error| <= 1e-5 x peak on x at equal iteration
counts; residuals within 1e-3 and the objective within 1e-4 relative."""

import numpy as np
import pytest

import oracle as O
from paper_2010_15491_amd import phantom, sr3d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = ELEM = 1e-5
LAM, MU = 2e-2, 5e-2


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def close(got, ref, tol=TOL, elem=ELEM):
    err = O.rel_l2(got, ref)
    worst = float(np.abs(np.asarray(got) - ref).max())
    assert err <= tol, f"rel-L2 {err:.3e}"
    assert worst <= elem * float(np.abs(ref).max()), f"max abs error {worst:.3e}"
    return err


def l1_problem(shape, rate, sigma, seed, frac=0.1, amp=1.0):
    p = phantom.make_problem(shape, rate, sigma, 0.01, seed, n_ellipsoids=8)
    psf = f32(p["psf"])
    y = O.degrade(p["x_true"], psf, rate) + p["noise"]
    y = f32(y + phantom.impulse_noise(y.shape, seed + 500, frac, amp))
    return y, psf, p["x_true"]


@pytest.mark.parametrize("shape,rate,sigma,mu_d,iters,aniso", [
    ((32, 32, 32), (2, 2, 2), 1.0, 1.0, 12, False),
    ((16, 32, 48), (2, 2, 4), 1.2, 2.0, 10, False),
    ((24, 32, 16), (4, 4, 2), 0.9, 0.5, 10, False),
    ((32, 24, 32), (2, 1, 2), 1.0, 1.0, 8, True),
    ((16, 16, 64), (1, 2, 2), 1.0, 1.0, 8, False),
])
def test_l1data_fixed_iterations_match_oracle(shape, rate, sigma, mu_d, iters, aniso):
    """Both x-update paths: the fused one (where its plan applies; with the
    m-axis R2C fused into the stencil at m = 64) and the fold on the natural
    spectrum (SR3D_UNFUSED)."""
    y, psf, _ = l1_problem(shape, rate, sigma, 80)
    flags = sr3d.FP64_REDUCE | sr3d.DATA_L1 | (sr3d.TV_ANISO if aniso else 0)
    ref = O.admm_l1data(y, psf, rate, LAM, MU, mu_d, iters, aniso=aniso)
    xs = {}
    for name, extra in (("default", 0), ("unfused", sr3d.UNFUSED)):
        print(f"l1 data {shape} {rate} mu_d {mu_d} aniso {aniso} {name}", flush=True)
        x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM, MU, iters, flags=flags | extra,
                             mu_data=mu_d)
        assert st.iters == iters and not st.converged
        err = close(host(x), ref.x)
        print(f"  rel-L2 {err:.2e}, primal {st.primal_rel:.4e} vs {ref.primal_rel:.4e}, "
              f"dual {st.dual_rel:.4e} vs {ref.dual_rel:.4e}")
        assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
        assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)
        assert np.isclose(st.objective,
                          O.l1data_objective(host(x), y, psf, rate, LAM, aniso=aniso), rtol=1e-4)
        xs[name] = host(x)
    close(xs["default"], xs["unfused"], tol=1e-6, elem=1e-6)


def test_l1data_warm_start_x0_fp32_reductions_and_graph():
    shape, rate, mu_d = (32, 32, 32), (2, 2, 2), 1.0
    y, psf, _ = l1_problem(shape, rate, 1.0, 81)
    x0 = f32(O.tikhonov(y, psf, rate, 1e-3))
    Y, P, X0 = dev(y), dev(psf), dev(x0)
    fl = sr3d.FP64_REDUCE | sr3d.DATA_L1
    x, st = sr3d.tv_admm(Y, P, rate, LAM, MU, 10, x0=X0, flags=fl, mu_data=mu_d)
    ref = O.admm_l1data(y, psf, rate, LAM, MU, mu_d, 10, x0=x0)
    close(host(x), ref.x)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)
    x32, _ = sr3d.tv_admm(Y, P, rate, LAM, MU, 10, x0=X0, flags=sr3d.DATA_L1, mu_data=mu_d)
    assert torch.equal(x, x32)  # the reductions do not feed back into x
    xg, sg = sr3d.tv_admm(Y, P, rate, LAM, MU, 10, x0=X0, flags=fl | sr3d.USE_GRAPH,
                          mu_data=mu_d)
    assert torch.equal(x, xg) and sg.iters == 10


def test_l1data_tolerance_stop_matches_oracle():
    shape, rate, mu_d, tol = (32, 32, 32), (2, 2, 2), 1.0, 2e-2
    y, psf, _ = l1_problem(shape, rate, 1.0, 82)
    ref = O.admm_l1data(y, psf, rate, LAM, MU, mu_d, 300, tol=tol)
    assert ref.converged and ref.iters > 5
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM, MU, 300, tol=tol,
                         flags=sr3d.FP64_REDUCE | sr3d.DATA_L1, mu_data=mu_d)
    print(f"stop at {st.iters} (oracle {ref.iters})")
    assert st.converged and abs(st.iters - ref.iters) <= 1
    assert st.primal_rel <= tol and st.dual_rel <= tol
    close(host(x), O.admm_l1data(y, psf, rate, LAM, MU, mu_d, st.iters).x)


def test_l1data_rejects_impulses_on_the_gpu():
    """With impulses on 10% of the LR voxels the l1 data term lands closer to
    the clean phantom than Algorithm 1's l2 data term at the same lam."""
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, xt = l1_problem(shape, rate, 1.0, 83, frac=0.1, amp=2.0)
    Y, P = dev(y), dev(psf)
    x1, _ = sr3d.tv_admm(Y, P, rate, 3e-2, MU, 200, flags=sr3d.FP64_REDUCE | sr3d.DATA_L1,
                         mu_data=1.0)
    x2, _ = sr3d.tv_admm(Y, P, rate, 3e-2, MU, 200)
    e1, e2 = O.rel_l2(host(x1), xt), O.rel_l2(host(x2), xt)
    print(f"distance to the clean phantom: l1 {e1:.3f}, l2 {e2:.3f}")
    assert e1 < 0.7 * e2
