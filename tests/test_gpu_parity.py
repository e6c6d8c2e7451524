"""GPU (HIP, through the C ABI) against the FP64 oracle, element by element.

Inputs are seeded synthetic phantoms; both sides get the same float32-rounded
y, PSF and x0. Bar for the FP32 path: rel-L2 <= 1e-5 against FP64.
"""

import time

import numpy as np
import pytest

import oracle as O
from paper_2010_15491_amd import phantom, sr3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-5
# Element-wise bar: max |x - x_ref| <= ELEM * max |x_ref|. A global rel-L2
# alone would let a large error at a few voxels pass (at 256^3 one voxel is
# 1/4096 of the norm); this bounds every voxel by the same 1e-5 taken
# relative to the volume's peak.
ELEM = 1e-5


def dev(a):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def progress(request, msg):
    """Prints a progress line past pytest's output capture (long oracle runs)."""
    capman = request.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        print(msg, flush=True)


def close(got, ref, tol=TOL, elem=ELEM):
    """Asserts rel-L2(got, ref) <= tol and max|got - ref| <= elem * max|ref|;
    returns the rel-L2 error."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    err = O.rel_l2(got, ref)
    peak = float(np.abs(ref).max())
    worst = float(np.abs(got - ref).max())
    assert err <= tol, f"rel-L2 {err:.3e} > {tol:.0e}"
    assert worst <= elem * peak, f"max abs error {worst:.3e} > {elem:.0e} x peak {peak:.3e}"
    return err


def problem(shape, rate, sigma, noise, seed, texture=False, n_ell=12):
    p = phantom.make_problem(shape, rate, sigma, noise, seed, texture=texture, n_ellipsoids=n_ell)
    psf = f32(p["psf"])
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    return y, psf, p["x_true"]


# ---------------------------------------------------------------------------
# FFT
# ---------------------------------------------------------------------------

LENGTHS = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024]


def fft_shapes():
    out = []
    for L in LENGTHS:
        out += [(L, 3, 4), (3, L, 6), (4, 3, L)]
    out += [(24, 48, 32), (8, 96, 64), (64, 64, 64), (16, 12, 2), (2, 768, 6), (1024, 2, 2)]
    return out


@pytest.mark.parametrize("shape", fft_shapes())
def test_rfft3d_matches_numpy(shape):
    rng = np.random.default_rng(sum(shape))
    x = f32(rng.standard_normal(shape))
    X = sr3d.rfft3d(dev(x))
    ref = np.fft.rfftn(x)
    got = X.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 2e-6, (shape, err)
    back = host(sr3d.irfft3d(X, shape))
    assert np.linalg.norm(back - x) / np.linalg.norm(x) < 2e-6


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_every_fft_tile_variant_is_correct(variant, tmp_path):
    """Force one tile variant for every kind and length, check the transforms."""
    f = tmp_path / "tiles.txt"
    f.write_text("".join(f"{k} {L} {variant}\n" for k in range(6) for L in LENGTHS))
    assert sr3d.tune_load(f) == 6 * len(LENGTHS)
    try:
        for shape in [(24, 48, 32), (8, 96, 64), (64, 64, 64), (3, 768, 6), (1024, 3, 4),
                      (4, 3, 1024), (12, 6, 3)]:
            rng = np.random.default_rng(sum(shape) + variant)
            x = f32(rng.standard_normal(shape))
            X = sr3d.rfft3d(dev(x))
            ref = np.fft.rfftn(x)
            got = X.cpu().numpy().astype(np.complex128)
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 2e-6, shape
            back = host(sr3d.irfft3d(X, shape))
            assert np.linalg.norm(back - x) / np.linalg.norm(x) < 2e-6, shape
    finally:
        f.write_text("".join(f"{k} {L} 1\n" for k in range(6) for L in LENGTHS))
        sr3d.tune_load(f)


def test_autotune_runs_and_keeps_results_correct():
    sr3d.autotune([((32, 48, 64), (2, 2, 4)), ((16, 16, 16), (2, 2, 2))], force=True)
    y, psf, _ = problem((32, 48, 64), (2, 2, 4), 1.2, 0.02, 3)
    x, st = sr3d.tv_admm(dev(y), dev(psf), (2, 2, 4), LAM_TV, MU, 5)
    ref = O.admm_tv(y, psf, (2, 2, 4), LAM_TV, MU, 5)
    close(host(x), ref.x)


def test_rfft3d_matches_bruteforce_dft():
    rng = np.random.default_rng(3)
    shape = (3, 4, 6)
    x = f32(rng.standard_normal(shape))
    S, N, M = shape
    s, n, m = np.meshgrid(np.arange(S), np.arange(N), np.arange(M), indexing="ij")
    ref = np.zeros((S, N, M // 2 + 1), complex)
    for ks in range(S):
        for kn in range(N):
            for km in range(M // 2 + 1):
                ref[ks, kn, km] = np.sum(x * np.exp(-2j * np.pi * (ks * s / S + kn * n / N + km * m / M)))
    got = sr3d.rfft3d(dev(x)).cpu().numpy()
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# Forward model and Tikhonov (eq. (12))
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("shape,rate,kshape", [((32, 32, 32), (2, 2, 2), (5, 5, 5)),
                                               ((16, 24, 48), (2, 3, 4), (3, 2, 5)),
                                               ((8, 96, 64), (4, 4, 2), (5, 3, 3))])
def test_degrade_matches_oracle(shape, rate, kshape):
    rng = np.random.default_rng(7)
    x = f32(rng.standard_normal(shape))
    psf = f32(rng.uniform(0.1, 1, kshape))
    psf /= psf.sum()
    psf = f32(psf)
    got = host(sr3d.degrade(dev(x), dev(psf), rate))
    ref = O.degrade(x, psf, rate)
    close(got, ref, tol=2e-6)


def test_tikhonov_config_32cube():
    """Plain Tikhonov closed form: 32^3, d = 2x2x2, PSF 5^3 sigma 1.0, noise 0.01, tau 1e-3."""
    y, psf, _ = problem((32, 32, 32), (2, 2, 2), 1.0, 0.01, 0)
    x = host(sr3d.tikhonov(dev(y), dev(psf), (2, 2, 2), 1e-3))
    ref = O.tikhonov(y, psf, (2, 2, 2), 1e-3)
    close(x, ref)


@pytest.mark.parametrize("shape,rate,kshape,lam", [
    ((32, 32, 32), (2, 2, 2), (3, 2, 5), 1e-3),
    ((16, 24, 48), (2, 3, 4), (3, 3, 3), 5e-3),
    ((48, 32, 24), (1, 1, 1), (5, 5, 5), 1e-2),
    ((8, 96, 64), (4, 4, 2), (5, 3, 3), 1e-3),
    ((64, 64, 32), (1, 2, 4), (7, 7, 7), 2e-3),
    ((12, 6, 3), (3, 2, 1), (3, 3, 3), 1e-2),
])
def test_tikhonov_matches_oracle_with_xbar(shape, rate, kshape, lam):
    rng = np.random.default_rng(11)
    psf = f32(rng.uniform(0.05, 1, kshape))
    psf = f32(psf / psf.sum())
    x_true = rng.standard_normal(shape)
    y = f32(O.degrade(x_true, psf, rate) + 0.01 * rng.standard_normal(O.lr_shape_of(shape, rate)))
    xbar = f32(rng.standard_normal(shape) * 0.1)
    got = host(sr3d.tikhonov(dev(y), dev(psf), rate, lam, xbar=dev(xbar)))
    ref = O.tikhonov(y, psf, rate, lam, xbar)
    close(got, ref)
    got0 = host(sr3d.tikhonov(dev(y), dev(psf), rate, lam))
    close(got0, O.tikhonov(y, psf, rate, lam))


# ---------------------------------------------------------------------------
# TV-ADMM (Algorithm 1)
# ---------------------------------------------------------------------------

LAM_TV, MU = 2e-3, 5e-2


@pytest.mark.parametrize("shape,rate,sigma,iters", [
    ((32, 32, 32), (2, 2, 2), 1.5, 1),
    ((32, 32, 32), (2, 2, 2), 1.5, 10),
    ((64, 64, 64), (2, 2, 2), 1.5, 100),
    ((32, 48, 64), (2, 2, 4), 1.2, 30),
    ((64, 96, 96), (4, 4, 2), 1.0, 20),
    ((24, 12, 16), (1, 1, 1), 1.0, 15),
])
def test_tv_admm_fixed_iterations_match_oracle(shape, rate, sigma, iters):
    y, psf, _ = problem(shape, rate, sigma, 0.02, 1)
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, iters)
    x = host(x)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, iters)
    assert st.iters == iters and not st.converged
    err = close(x, ref.x)
    print(f"{shape} {rate} {iters} it: rel-L2 {err:.3e}, primal {st.primal_rel:.4e} vs "
          f"{ref.primal_rel:.4e}, dual {st.dual_rel:.4e} vs {ref.dual_rel:.4e}")
    assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)


def test_tv_admm_warm_start_x0_matches_oracle():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, x_true = problem(shape, rate, 1.5, 0.02, 5)
    x0 = f32(O.tikhonov(y, psf, rate, 1e-3))
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 25, x0=dev(x0))
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 25, x0=x0)
    close(host(x), ref.x)


def test_tv_admm_dual_warm_start_matches_oracle():
    shape, rate = (32, 32, 48), (2, 2, 2)
    y, psf, x_true = problem(shape, rate, 1.5, 0.02, 12)
    x0 = f32(O.tikhonov(y, psf, rate, 1e-3))
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 10, x0=dev(x0),
                         flags=sr3d.FP64_REDUCE | sr3d.WARM_DUAL)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 10, x0=x0, warm_dual=True)
    close(host(x), ref.x)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)


def test_tv_admm_separate_dual_tolerance_matches_oracle():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 13)
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 150, tol=2e-3, tol_dual=5e-2)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 150, tol=2e-3, tol_dual=5e-2)
    assert ref.converged and st.converged and abs(st.iters - ref.iters) <= 1
    assert st.primal_rel <= 2e-3 and st.dual_rel <= 5e-2


def test_tv_admm_tolerance_stop_matches_oracle():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 6)
    tol = 2e-2
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 200, tol=tol)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 200, tol=tol)
    assert ref.converged and st.converged
    assert abs(st.iters - ref.iters) <= 1
    assert st.primal_rel <= tol and st.dual_rel <= tol


def test_tv_admm_objective_matches_oracle():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 7)
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 12)
    obj = O.tv_objective(host(x), y, psf, rate, LAM_TV)
    assert np.isclose(st.objective, obj, rtol=1e-4)


def test_tv_admm_state_invariants_and_resume():
    """||d_j|| <= lam/mu with d = nu - shrink(nu); resuming from the state
    continues the same iteration sequence."""
    shape, rate = (32, 32, 64), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 8)
    N = int(np.prod(shape))
    state = torch.zeros(3 * N, device="cuda")
    x10, _ = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 10, state=state)
    nu = host(state).reshape((3,) + shape)
    u = O.shrink(nu, LAM_TV / MU)
    d = nu - u
    assert np.sqrt((d ** 2).sum(0)).max() <= (LAM_TV / MU) * (1 + 1e-5)
    x20r, _ = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 10, state=state,
                           flags=sr3d.FP64_REDUCE | sr3d.RESUME)
    x20, _ = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 20)
    assert torch.equal(x20r, x20)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 20)
    close(host(x20), ref.x)


def test_fp32_and_fp64_reductions_leave_x_unchanged_and_graph_replay():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 9)
    Y, P = dev(y), dev(psf)
    xa, sa = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 17, flags=sr3d.FP64_REDUCE)
    xb, sb = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 17, flags=0)
    xc, sc = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 17,
                          flags=sr3d.FP64_REDUCE | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(5))
    assert torch.equal(xa, xb) and torch.equal(xa, xc)
    assert sa.iters == sb.iters == sc.iters == 17
    assert np.isclose(sa.primal_rel, sb.primal_rel, rtol=1e-3)


def test_repeat_runs_are_bitwise_identical():
    shape, rate = (32, 32, 32), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 10)
    a, sa = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 9)
    b, sb = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 9)
    assert torch.equal(a, b) and sa.primal_rel == sb.primal_rel


def test_singular_lambda0_is_reported():
    shape, rate = (16, 16, 16), (2, 2, 2)
    y = np.zeros(O.lr_shape_of(shape, rate))
    psf = np.array([[[1.0, -1.0]]])  # sums to zero: Lambda(0) = 0
    with pytest.raises(sr3d.Sr3dError) as e:
        sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 3)
    assert e.value.status == -6


def test_nonfinite_input_is_reported():
    shape, rate = (16, 16, 16), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.0, 0.02, 11, n_ell=3)
    y[1, 2, 3] = np.nan
    with pytest.raises(sr3d.Sr3dError) as e:
        sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 3)
    assert e.value.status == -7


def test_batch_matches_single_solves():
    cases = [((32, 32, 32), (2, 2, 2), 1.0), ((32, 48, 48), (4, 4, 2), 1.5),
             ((16, 32, 32), (2, 2, 4), 0.8)]
    probs, refs = [], []
    for i, (shape, rate, sig) in enumerate(cases):
        y, psf, _ = problem(shape, rate, sig, 0.02, 100 + i, n_ell=6)
        probs.append(dict(y=dev(y), psf=dev(psf), rate=rate, lam=LAM_TV, mu=MU, max_iter=15,
                          tol=0.0))
        refs.append(O.admm_tv(y, psf, rate, LAM_TV, MU, 15).x)
    xs, sts = sr3d.batch(probs)
    for x, st, ref, q in zip(xs, sts, refs, probs):
        single, _ = sr3d.tv_admm(q["y"], q["psf"], q["rate"], LAM_TV, MU, 15)
        assert st.iters == 15
        close(host(x), host(single), tol=1e-6)
        close(host(x), ref)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_uneven_volumes_stop_like_single_solves(graph):
    """Uneven sizes and rates; each volume stops at its own iteration, exactly
    as its single solve does, and returns the same x."""
    cases = [((64, 64, 64), (2, 2, 2), 1.0), ((64, 96, 96), (4, 4, 2), 1.5),
             ((32, 48, 48), (2, 2, 4), 0.8), ((32, 32, 32), (2, 2, 2), 2.0),
             ((24, 12, 16), (1, 1, 1), 1.0)]
    tol = 3e-2  # the oracle stops these at 47, 50, 46, >120 (cap) and 56 iterations
    probs, singles = [], []
    for i, (shape, rate, sig) in enumerate(cases):
        y, psf, _ = problem(shape, rate, sig, 0.02, 200 + i, n_ell=6)
        q = dict(y=dev(y), psf=dev(psf), rate=rate, lam=LAM_TV, mu=MU, max_iter=120, tol=tol)
        probs.append(q)
        singles.append(sr3d.tv_admm(q["y"], q["psf"], rate, LAM_TV, MU, 120, tol=tol))
    flags = sr3d.FP64_REDUCE | (sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(4) if graph else 0)
    xs, sts = sr3d.batch(probs, flags=flags)
    iters = [st.iters for st in sts]
    assert len(set(iters)) > 1, iters  # volumes really stop at different iterations
    for x, st, (xs1, st1) in zip(xs, sts, singles):
        assert st.iters == st1.iters and st.converged == st1.converged
        close(host(x), host(xs1), tol=1e-6)


# ---------------------------------------------------------------------------
# Fused x-update (s-FFT + alias-group solve + inverse s-FFT in one kernel)
# against the separate kernels and the oracle, on geometries that exercise
# its unit structure: odd N_l, self-conjugate m classes, odd m, unequal class
# sizes, single-sample axes, and an s-length outside the fused set.
# ---------------------------------------------------------------------------


def fit_psf(psf, shape):
    """Central part of the PSF that fits the volume, renormalised to sum 1."""
    sl = tuple(slice((k - min(k, n)) // 2, (k - min(k, n)) // 2 + min(k, n))
               for k, n in zip(psf.shape, shape))
    q = psf[sl]
    return f32(q / q.sum())


FUSE_CASES = [
    ((16, 12, 12), (3, 4, 2)),
    ((32, 16, 6), (3, 2, 2)),
    ((48, 8, 3), (1, 1, 3)),
    ((24, 6, 8), (4, 3, 1)),
    ((32, 1, 32), (2, 1, 2)),
    ((32, 16, 1), (1, 2, 2)),
    ((8, 16, 16), (2, 2, 2)),
    ((64, 32, 32), (2, 2, 4)),
    ((512, 8, 8), (2, 2, 2)),
    ((384, 8, 8), (2, 2, 4)),
    ((192, 24, 24), (2, 2, 2)),
    ((128, 32, 32), (4, 4, 2)),
    # d = 8 at rates other than 2 x 2 x 2 (the general 8-member instance)
    ((32, 16, 16), (1, 2, 4)),
    ((16, 16, 32), (4, 2, 1)),
    # s = 96 at every compile-time group size (d = 8, 16, 32)
    ((96, 24, 24), (2, 2, 2)),
    ((96, 16, 16), (2, 2, 4)),
    ((96, 32, 32), (4, 4, 2)),
]


@pytest.mark.parametrize("shape,rate", FUSE_CASES)
def test_fused_and_unfused_x_update_match_oracle(shape, rate):
    p = phantom.make_problem(shape, rate, 1.0, 0.02, 21, n_ellipsoids=6)
    psf = fit_psf(p["psf"], shape)
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 8)
    xf, sf = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 8)
    xu, su = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 8,
                          flags=sr3d.FP64_REDUCE | sr3d.UNFUSED)
    ef, eu = close(host(xf), ref.x), close(host(xu), ref.x)
    print(f"{shape} {rate}: fused {ef:.2e}, unfused {eu:.2e}")
    assert np.isclose(sf.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(sf.dual_rel, ref.dual_rel, rtol=1e-3)
    close(host(xf), host(xu), tol=1e-6)
    assert np.isclose(sf.primal_rel, su.primal_rel, rtol=1e-4)
    assert np.isclose(sf.objective, su.objective, rtol=1e-5)
    assert np.isclose(sf.objective, O.tv_objective(host(xf), y, psf, rate, LAM_TV), rtol=1e-4)


# Row lengths the stencil with the fused m-axis R2C takes (64 .. 256), with
# n-lengths that leave a ragged last tile of rows (n = 1, 2, 3, 6) or none;
# m = 384 and 512 take the separate kernels whatever the flags.
ROW_CASES = [
    ((16, 6, 64), (2, 2, 2)),
    ((24, 12, 64), (1, 3, 3)),
    ((32, 3, 128), (2, 1, 2)),
    ((16, 1, 256), (2, 1, 2)),
    ((16, 2, 192), (2, 2, 2)),
    ((16, 8, 384), (4, 2, 2)),
    ((16, 4, 512), (2, 2, 2)),
]


@pytest.mark.parametrize("shape,rate", ROW_CASES)
def test_fused_stencil_r2c_matches_separate_kernels(shape, rate):
    """The stencil with the next x-update's m-axis R2C fused in gives the same
    bits as the separate stencil and R2C kernels, eagerly and under graph
    replay, and the oracle's iterate."""
    p = phantom.make_problem(shape, rate, 1.0, 0.02, 31, n_ellipsoids=6)
    psf = fit_psf(p["psf"], shape)
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    Y, P = dev(y), dev(psf)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 7)
    xf, sf = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 7)
    xs, ss = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 7,
                          flags=sr3d.FP64_REDUCE | sr3d.SEPARATE_R2C)
    xg, sg = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 7,
                          flags=sr3d.FP64_REDUCE | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(3))
    print(f"{shape} {rate}: {O.rel_l2(host(xf), ref.x):.2e}")
    assert torch.equal(xf, xs) and torch.equal(xf, xg)
    assert sf.iters == ss.iters == sg.iters == 7
    close(host(xf), ref.x)
    # residual sums over a different tiling: equal up to FP32 summation order
    assert np.isclose(sf.primal_rel, ss.primal_rel, rtol=1e-4)
    assert np.isclose(sf.dual_rel, ss.dual_rel, rtol=1e-4)
    assert np.isclose(sf.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(sf.dual_rel, ref.dual_rel, rtol=1e-3)


def test_fused_stencil_r2c_tolerance_stop_matches_oracle():
    """The stopping test carried by the n pass stops where the oracle does."""
    shape, rate = (32, 32, 64), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 14)
    tol = 2e-2
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 200, tol=tol)
    for flags in (sr3d.FP64_REDUCE, sr3d.FP64_REDUCE | sr3d.CHECK_INTERVAL(1),
                  sr3d.FP64_REDUCE | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(4)):
        x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 200, tol=tol, flags=flags)
        assert ref.converged and st.converged and abs(st.iters - ref.iters) <= 1
        assert st.primal_rel <= tol and st.dual_rel <= tol
        close(host(x), O.admm_tv(y, psf, rate, LAM_TV, MU, st.iters).x)


# Anisotropic TV through the same x-step: fused stencil (m = 64, 128), tiled
# stencil (m = 32, 24 and SR3D_SEPARATE_R2C), unfused x-update.
ANISO_CASES = [
    ((32, 32, 32), (2, 2, 2), 0),
    ((16, 6, 64), (2, 2, 2), 0),
    ((32, 3, 128), (2, 1, 2), 0),
    ((32, 32, 64), (2, 2, 2), 0x40),
    ((24, 12, 24), (1, 3, 3), 0x20),
]


@pytest.mark.parametrize("shape,rate,extra", ANISO_CASES)
def test_tv_aniso_matches_oracle(shape, rate, extra):
    p = phantom.make_problem(shape, rate, 1.0, 0.02, 41, n_ellipsoids=6)
    psf = fit_psf(p["psf"], shape)
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 10, aniso=True)
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 10,
                         flags=sr3d.FP64_REDUCE | sr3d.TV_ANISO | extra)
    err = close(host(x), ref.x)
    print(f"{shape} {rate} flags+{extra:#x}: aniso rel-L2 {err:.2e}")
    assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)
    assert np.isclose(st.objective, O.tv_objective(host(x), y, psf, rate, LAM_TV, aniso=True),
                      rtol=1e-4)
    iso = O.admm_tv(y, psf, rate, LAM_TV, MU, 10)
    assert O.rel_l2(iso.x, ref.x) > 100 * TOL  # the two regularisers really differ here


def test_tv_aniso_paths_agree_bitwise_and_resume():
    shape, rate = (32, 32, 64), (2, 2, 2)
    y, psf, _ = problem(shape, rate, 1.5, 0.02, 42)
    Y, P = dev(y), dev(psf)
    fl = sr3d.FP64_REDUCE | sr3d.TV_ANISO
    xf, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 12, flags=fl)
    xs, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 12, flags=fl | sr3d.SEPARATE_R2C)
    xg, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 12, flags=fl | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(5))
    assert torch.equal(xf, xs) and torch.equal(xf, xg)
    state = torch.zeros(3 * y.size * 8, device="cuda")
    sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 6, state=state, flags=fl)
    xr, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 6, state=state, flags=fl | sr3d.RESUME)
    assert torch.equal(xr, xf)
    # the state carries the anisotropic dual: |d_a| <= lam/mu per component
    nu = host(state).reshape((3,) + shape)
    assert np.abs(nu - O.shrink_aniso(nu, LAM_TV / MU)).max() <= (LAM_TV / MU) * (1 + 1e-5)


def test_tv_aniso_batch_matches_single_solves():
    cases = [((32, 32, 32), (2, 2, 2)), ((16, 6, 64), (2, 2, 2)), ((24, 12, 24), (1, 3, 3))]
    fl = sr3d.FP64_REDUCE | sr3d.TV_ANISO
    probs, refs = [], []
    for i, (shape, rate) in enumerate(cases):
        p = phantom.make_problem(shape, rate, 1.0, 0.02, 400 + i, n_ellipsoids=6)
        psf = fit_psf(p["psf"], shape)
        y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
        probs.append(dict(y=dev(y), psf=dev(psf), rate=rate, lam=LAM_TV, mu=MU, max_iter=9,
                          tol=0.0))
        refs.append(O.admm_tv(y, psf, rate, LAM_TV, MU, 9, aniso=True).x)
    xs, sts = sr3d.batch(probs, flags=fl)
    for x, st, ref, q in zip(xs, sts, refs, probs):
        single, _ = sr3d.tv_admm(q["y"], q["psf"], q["rate"], LAM_TV, MU, 9, flags=fl)
        assert st.iters == 9
        close(host(x), host(single), tol=1e-6)
        close(host(x), ref)


# l1 of orthonormal 3D Haar details through the same x-step (Tikhonov fold).
WAVELET_CASES = [
    ((16, 16, 16), (1, 1, 1), 1),
    ((32, 32, 32), (2, 2, 2), 1),
    ((32, 16, 32), (2, 1, 2), 2),
    ((16, 16, 32), (1, 1, 1), 3),
    ((24, 24, 48), (2, 2, 2), 3),
    ((16, 16, 96), (2, 2, 2), 2),
    ((16, 32, 32), (1, 1, 1), 4),
]


@pytest.mark.parametrize("unfused", [False, True])
@pytest.mark.parametrize("shape,rate,levels", WAVELET_CASES)
def test_wavelet_l1_matches_oracle(shape, rate, levels, unfused):
    """The Tikhonov x-step through the fused x-update kernel (A = mu at every
    member) and through the unfused fold."""
    y, psf, _ = problem(shape, rate, 1.0, 0.02, 51, n_ell=6)
    ref = O.admm_wavelet(y, psf, rate, LAM_TV, MU, 10, levels=levels)
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 10,
                         flags=sr3d.FP64_REDUCE | sr3d.REG_HAAR | sr3d.HAAR_LEVELS(levels)
                         | (sr3d.UNFUSED if unfused else 0))
    err = close(host(x), ref.x)
    print(f"{shape} {rate} levels {levels} unfused {unfused}: rel-L2 {err:.2e}")
    assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)
    assert np.isclose(st.objective, O.wavelet_objective(host(x), y, psf, rate, LAM_TV, levels),
                      rtol=1e-4)


def test_wavelet_l1_resume_graph_and_tolerance_stop():
    shape, rate, levels = (16, 16, 32), (1, 1, 1), 2
    y, psf, _ = problem(shape, rate, 1.0, 0.02, 52, n_ell=6)
    Y, P = dev(y), dev(psf)
    fl = sr3d.FP64_REDUCE | sr3d.REG_HAAR | sr3d.HAAR_LEVELS(levels)
    x12, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 12, flags=fl)
    xg, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 12, flags=fl | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(5))
    assert torch.equal(x12, xg)
    state = torch.zeros(3 * y.size, device="cuda")
    sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 7, state=state, flags=fl)
    xr, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 5, state=state, flags=fl | sr3d.RESUME)
    assert torch.equal(xr, x12)
    # warm start: nu0 = W x0
    x0 = f32(O.tikhonov(y, psf, rate, 1e-3))
    xw, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 6, x0=dev(x0), flags=fl)
    close(host(xw), O.admm_wavelet(y, psf, rate, LAM_TV, MU, 6, x0=x0, levels=levels).x)
    tol = 1e-3
    ref = O.admm_wavelet(y, psf, rate, LAM_TV, MU, 300, tol=tol, levels=levels)
    x, st = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 300, tol=tol, flags=fl | sr3d.CHECK_INTERVAL(1))
    assert ref.converged and st.converged and abs(st.iters - ref.iters) <= 1
    close(host(x), O.admm_wavelet(y, psf, rate, LAM_TV, MU, st.iters, levels=levels).x)


@pytest.mark.parametrize("extra", [0, 0x20, 0x40])
def test_batch_mixes_fused_and_unfused_volumes(extra):
    """Default (fused x-update, fused stencil where m allows), SR3D_UNFUSED and
    SR3D_SEPARATE_R2C, over volumes that take different kernels."""
    cases = [((8, 32, 32), (2, 2, 2)), ((32, 32, 32), (2, 2, 2)), ((16, 12, 12), (3, 4, 2)),
             ((24, 6, 8), (4, 3, 1)), ((16, 8, 64), (2, 2, 2)), ((32, 6, 128), (2, 2, 2))]
    flags = sr3d.FP64_REDUCE | extra
    probs, refs = [], []
    for i, (shape, rate) in enumerate(cases):
        p = phantom.make_problem(shape, rate, 1.0, 0.02, 300 + i, n_ellipsoids=6)
        psf = fit_psf(p["psf"], shape)
        y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
        probs.append(dict(y=dev(y), psf=dev(psf), rate=rate, lam=LAM_TV, mu=MU, max_iter=12,
                          tol=0.0))
        refs.append(O.admm_tv(y, psf, rate, LAM_TV, MU, 12).x)
    xs, sts = sr3d.batch(probs, flags=flags)
    for x, st, ref, q in zip(xs, sts, refs, probs):
        single, s1 = sr3d.tv_admm(q["y"], q["psf"], q["rate"], LAM_TV, MU, 12, flags=flags)
        assert st.iters == 12
        close(host(x), host(single), tol=1e-6)
        close(host(x), ref)


# ---------------------------------------------------------------------------
# Full size (256^3, the benchmark workload): first iterate against the oracle,
# invariants after the benchmark's iterations.
# ---------------------------------------------------------------------------


def test_full_size_256_first_iterations_and_invariants():
    shape, rate = (256, 256, 256), (2, 2, 2)
    p = phantom.make_problem(shape, rate, 1.5, 0.02, 1, texture=True)
    psf = f32(p["psf"])
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    Y, P = dev(y), dev(psf)
    x2, _ = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 2)
    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 2)
    err = close(host(x2), ref.x)
    print(f"256^3 after 2 iterations: rel-L2 {err:.3e}")
    state = torch.zeros(3 * y.size * 8, device="cuda")
    x, st = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 200, tol=1e-4, state=state)
    nu = host(state).reshape((3,) + shape)
    d = nu - O.shrink(nu, LAM_TV / MU)
    assert np.sqrt((d ** 2).sum(0)).max() <= (LAM_TV / MU) * (1 + 1e-5)
    assert np.isfinite(st.objective) and st.iters >= 1
    print(f"256^3 stop: iters {st.iters} converged {st.converged} "
          f"primal {st.primal_rel:.3e} dual {st.dual_rel:.3e}")
    # the benchmark's kernels (stencil with the fused R2C, fused x-update)
    # against the separate stencil + R2C and the unfused x-update
    xf, sf = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 5)
    xs, ss = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 5, flags=sr3d.FP64_REDUCE | sr3d.SEPARATE_R2C)
    xu, su = sr3d.tv_admm(Y, P, rate, LAM_TV, MU, 5, flags=sr3d.FP64_REDUCE | sr3d.UNFUSED)
    assert torch.equal(xf, xs)
    close(host(xf), host(xu), tol=1e-6)
    for a_, b_ in ((sf, ss), (sf, su)):
        assert np.isclose(a_.primal_rel, b_.primal_rel, rtol=1e-4)
        assert np.isclose(a_.dual_rel, b_.dual_rel, rtol=1e-4)


def test_batch_with_96x192x192_volumes_at_every_group_size():
    """The batch workload's largest s = 96 volumes (96 x 192 x 192 at d = 8, 16
    and 32) through sr3d_batch, each against the oracle: the fused x-update at
    s = 96 for every compile-time group size and the batched fused stencil at
    m = 192."""
    cases = [((96, 192, 192), (4, 4, 2), 1.2), ((96, 192, 192), (2, 2, 4), 0.9),
             ((96, 192, 192), (2, 2, 2), 1.6), ((64, 64, 64), (2, 2, 2), 1.0)]
    probs, refs = [], []
    for i, (shape, rate, sig) in enumerate(cases):
        y, psf, _ = problem(shape, rate, sig, 0.02, 500 + i)
        probs.append(dict(y=dev(y), psf=dev(psf), rate=rate, lam=LAM_TV, mu=MU, max_iter=10,
                          tol=0.0))
        refs.append(O.admm_tv(y, psf, rate, LAM_TV, MU, 10))
    xs, sts = sr3d.batch(probs, flags=sr3d.FP64_REDUCE)
    for (shape, rate, _), x, st, ref in zip(cases, xs, sts, refs):
        assert st.iters == 10
        err = close(host(x), ref.x)
        print(f"batch {shape} {rate}: rel-L2 {err:.2e}")
        assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
        assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)


@pytest.mark.timeout(1800)
def test_full_size_256_benchmark_solve_matches_oracle(request):
    """The benchmark's solve exactly (256^3, seed 1 with texture, d = 2x2x2,
    sigma 1.5, lambda 2e-3, mu 5e-2, tol 1e-4, cap 200, FP64 reductions, the
    default kernels) against the oracle's Algorithm 1 with the same stopping
    rule: same iteration count and stop decision, x within the bar."""
    shape, rate = (256, 256, 256), (2, 2, 2)
    p = phantom.make_problem(shape, rate, 1.5, 0.02, 1, texture=True)
    psf = f32(p["psf"])
    y = f32(O.degrade(p["x_true"], psf, rate) + p["noise"])
    x, st = sr3d.tv_admm(dev(y), dev(psf), rate, LAM_TV, MU, 200, tol=1e-4,
                         flags=sr3d.FP64_REDUCE)
    xg = host(x)
    del x
    progress(request, f"GPU 256^3 solve: {st.iters} iterations, converged {st.converged}; "
                      "oracle running")
    t0 = time.perf_counter()

    def cb(it, *_):
        if it % 20 == 0:
            progress(request, f"oracle 256^3 iteration {it}/200, {time.perf_counter() - t0:.0f} s")

    ref = O.admm_tv(y, psf, rate, LAM_TV, MU, 200, tol=1e-4, callback=cb)
    err = close(xg, ref.x)
    worst = float(np.abs(xg - ref.x).max() / np.abs(ref.x).max())
    progress(request, f"256^3 x 200: rel-L2 {err:.3e}, max abs error / peak {worst:.3e}, "
                      f"iters {st.iters}/{ref.iters}, primal {st.primal_rel:.5e} vs "
                      f"{ref.primal_rel:.5e}, dual {st.dual_rel:.5e} vs {ref.dual_rel:.5e}")
    assert st.iters == ref.iters and bool(st.converged) == ref.converged
    assert np.isclose(st.primal_rel, ref.primal_rel, rtol=1e-3)
    assert np.isclose(st.dual_rel, ref.dual_rel, rtol=1e-3)
    assert np.isclose(st.objective, O.tv_objective(xg, y, psf, rate, LAM_TV), rtol=1e-5)
