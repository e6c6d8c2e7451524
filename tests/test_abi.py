"""C-ABI checks that need no GPU: the library loads, exports every function
include/sr3d.h declares, and rejects bad arguments on the host before any HIP
call (status codes of the header)."""

import ctypes
import os
import re

import pytest

from paper_2010_15491_amd import sr3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sr3d.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr3d_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(sr3d.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = sr3d.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = sr3d.load()
    for code, name in sr3d.STATUS.items():
        assert lib.sr3d_status_string(code).decode() == name


def _prob(hr=(32, 32, 32), rate=(2, 2, 2), psf=(5, 5, 5), lam=1e-3, mu=5e-2, tol=0.0, it=10,
          ptr=1):
    p = sr3d.Problem()
    p.hr = sr3d.Dims(hr[2], hr[1], hr[0])
    p.rate = sr3d.Rate(*rate)
    p.psf_dims = sr3d.Dims(psf[2], psf[1], psf[0])
    p.y, p.psf, p.x = (None, None, None) if ptr is None else (ptr, ptr + 8, ptr + 16)
    p.lambda_tv, p.mu, p.tol, p.max_iter = lam, mu, tol, it
    return p


def test_workspace_size_query():
    lib = sr3d.load()
    p = _prob()
    n_tik = lib.sr3d_workspace_size(sr3d.OP_TIKHONOV, ctypes.byref(p), 1)
    n_tv = lib.sr3d_workspace_size(sr3d.OP_TV_ADMM, ctypes.byref(p), 1)
    assert n_tik > 4 * 32 ** 3 and n_tv > n_tik
    bad = _prob(hr=(30, 32, 32))
    assert lib.sr3d_workspace_size(sr3d.OP_TV_ADMM, ctypes.byref(bad), 1) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(hr=(32, 32, 33)), "SR3D_ERR_NOT_DIVISIBLE"),
    (dict(hr=(40, 40, 40)), "SR3D_ERR_UNSUPPORTED_SIZE"),
    (dict(hr=(32, 32, 2048), rate=(2, 2, 2)), "SR3D_ERR_UNSUPPORTED_SIZE"),
    (dict(rate=(8, 8, 4)), "SR3D_ERR_UNSUPPORTED_SIZE"),
    (dict(psf=(5, 5, 40)), "SR3D_ERR_PSF_TOO_LARGE"),
    (dict(lam=0.0), "SR3D_ERR_INVALID_ARG"),
    (dict(mu=-1.0), "SR3D_ERR_INVALID_ARG"),
    (dict(tol=-1.0), "SR3D_ERR_INVALID_ARG"),
    (dict(it=0), "SR3D_ERR_INVALID_ARG"),
    (dict(rate=(0, 2, 2)), "SR3D_ERR_INVALID_ARG"),
    (dict(ptr=None), "SR3D_ERR_INVALID_ARG"),
    (dict(), "SR3D_ERR_WORKSPACE"),
])
def test_tv_admm_host_argument_errors(kw, code):
    lib = sr3d.load()
    p = _prob(**kw)
    rc = lib.sr3d_tv_admm(ctypes.byref(p), 0, None, None, 0, None)
    assert sr3d.STATUS[rc] == code
    assert lib.sr3d_last_error().decode() != ""


def test_tikhonov_host_argument_errors():
    lib = sr3d.load()
    d, r, k = sr3d.Dims(32, 32, 32), sr3d.Rate(2, 2, 2), sr3d.Dims(5, 5, 5)
    assert lib.sr3d_tikhonov(d, r, 1, 1, k, None, 0.0, 2, None, 0, None) == -1
    assert lib.sr3d_tikhonov(d, r, None, 1, k, None, 1e-3, 2, None, 0, None) == -1
    assert lib.sr3d_tikhonov(d, r, 1, 1, k, None, 1e-3, 1, None, 0, None) == -1  # x aliases y
    assert lib.sr3d_tikhonov(sr3d.Dims(32, 32, 31), r, 1, 1, k, None, 1e-3, 2, None, 0, None) == -2
    assert lib.sr3d_tikhonov(d, r, 1, 1, k, None, 1e-3, 2, None, 0, None) == -5


def test_batch_and_resume_host_errors():
    lib = sr3d.load()
    arr = (sr3d.Problem * 2)(_prob(), _prob(hr=(32, 32, 31)))
    assert lib.sr3d_batch(arr, 2, 0, None, None, 0, None) == -2
    assert lib.sr3d_batch(arr, 0, 0, None, None, 0, None) == -1
    p = _prob()
    assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.RESUME, None, None, 0, None) == -1


def test_fft_host_errors():
    lib = sr3d.load()
    assert lib.sr3d_rfft3d(sr3d.Dims(40, 8, 8), 1, 2, None) == -4
    assert lib.sr3d_rfft3d(sr3d.Dims(32, 8, 8), None, 2, None) == -1
    assert lib.sr3d_irfft3d(sr3d.Dims(0, 8, 8), 1, 2, None) == -1


def _header_flags():
    text = open(os.path.join(ROOT, "include", "sr3d.h")).read()
    return {m.group(1): int(m.group(2), 16)
            for m in re.finditer(r"#define SR3D_([A-Z0-9_]+)\s+(0x[0-9a-fA-F]+)\b", text)}


def test_binding_flag_values_match_the_header():
    flags = _header_flags()
    for name in ("FP64_REDUCE", "RESUME", "USE_GRAPH", "PROFILE", "WARM_DUAL", "UNFUSED",
                 "SEPARATE_R2C", "TV_ANISO", "REG_HAAR", "DATA_L1"):
        assert getattr(sr3d, name) == flags[name], name
    # single bits, none inside the CHECK_INTERVAL (8-15) or HAAR_LEVELS (16-19) fields
    bits = [flags[n] for n in flags if n not in ("ERR_INVALID_ARG",)]
    for b in bits:
        assert b & (b - 1) == 0 and b & 0xFFF00 == 0, hex(b)
    assert sr3d.CHECK_INTERVAL(255) == 0xFF00 and sr3d.HAAR_LEVELS(15) == 0xF0000


def test_header_compiles_as_c():
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc")
    rocm_inc = "/opt/rocm/include"
    if not cc or not os.path.isdir(rocm_inc):
        pytest.skip("needs gcc and the ROCm headers")
    src = ('#include "sr3d.h"\n'
           "int f(void) { return SR3D_CHECK_INTERVAL(3) | SR3D_HAAR_LEVELS(2) | SR3D_REG_HAAR"
           " | SR3D_TV_ANISO | SR3D_SEPARATE_R2C | SR3D_DATA_L1; }\n")
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "h.c")
        with open(c, "w") as f:
            f.write(src)
        r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
                            "-I", os.path.join(ROOT, "include"), "-I", rocm_inc, "-c", c, "-o",
                            os.path.join(td, "h.o")], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_wavelet_host_argument_errors():
    lib = sr3d.load()
    lv2 = sr3d.REG_HAAR | sr3d.HAAR_LEVELS(2)
    p = _prob(hr=(32, 32, 6), rate=(2, 2, 2))  # m = 6 is no multiple of 4
    assert sr3d.STATUS[lib.sr3d_tv_admm(ctypes.byref(p), lv2, None, None, 0, None)] == \
        "SR3D_ERR_INVALID_ARG"
    p = _prob()
    assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.REG_HAAR | sr3d.TV_ANISO, None, None, 0,
                            None) == -1
    assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.REG_HAAR | sr3d.HAAR_LEVELS(9), None, None, 0,
                            None) == -1
    arr = (sr3d.Problem * 1)(_prob())
    assert lib.sr3d_batch(arr, 1, sr3d.REG_HAAR, None, None, 0, None) == -1


def test_tikhonov_noalloc_host_errors():
    """Beyond its static scratch, or with bad arguments, the allocation-free
    entry point fails on the host before any HIP call."""
    lib = sr3d.load()
    big = sr3d.Dims(256, 256, 256)
    rc = lib.sr3d_tikhonov_noalloc(big, sr3d.Rate(2, 2, 2), 1, 9, sr3d.Dims(7, 7, 7), None,
                                   1e-3, 17, None)
    assert sr3d.STATUS[rc] == "SR3D_ERR_WORKSPACE"
    assert "static scratch" in lib.sr3d_last_error().decode()
    small = sr3d.Dims(32, 32, 32)
    rc = lib.sr3d_tikhonov_noalloc(small, sr3d.Rate(2, 2, 2), None, 9, sr3d.Dims(5, 5, 5), None,
                                   1e-3, 17, None)
    assert sr3d.STATUS[rc] == "SR3D_ERR_INVALID_ARG"
    rc = lib.sr3d_tikhonov_noalloc(small, sr3d.Rate(2, 2, 2), 1, 9, sr3d.Dims(5, 5, 5), None,
                                   0.0, 17, None)
    assert sr3d.STATUS[rc] == "SR3D_ERR_INVALID_ARG"
    # the limit: a 128^3 solve fits the 64 MiB array, 256 x 128 x 128 does not
    p = _prob(hr=(128, 128, 128), psf=(7, 7, 7))
    assert lib.sr3d_workspace_size(sr3d.OP_TIKHONOV, ctypes.byref(p), 1) <= sr3d.NOALLOC_SCRATCH_BYTES
    p = _prob(hr=(256, 128, 128), psf=(7, 7, 7))
    assert lib.sr3d_workspace_size(sr3d.OP_TIKHONOV, ctypes.byref(p), 1) > sr3d.NOALLOC_SCRATCH_BYTES


def test_l1_data_host_argument_errors():
    """SR3D_DATA_L1 needs mu_data > 0 and excludes the Haar form, the dual
    warm start, resume and the batch; all rejected before any HIP call."""
    lib = sr3d.load()
    p = _prob()
    p.mu_data = 0.0
    assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.DATA_L1, None, None, 0, None) == -1
    assert "mu_data" in lib.sr3d_last_error().decode()
    p.mu_data = float("inf")
    assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.DATA_L1, None, None, 0, None) == -1
    p.mu_data = 1.0
    for extra in (sr3d.REG_HAAR, sr3d.WARM_DUAL, sr3d.RESUME):
        assert lib.sr3d_tv_admm(ctypes.byref(p), sr3d.DATA_L1 | extra, None, None, 0, None) == -1
    # valid arguments reach the workspace check
    assert sr3d.STATUS[lib.sr3d_tv_admm(ctypes.byref(p), sr3d.DATA_L1, None, None, 0, None)] == \
        "SR3D_ERR_WORKSPACE"
    arr = (sr3d.Problem * 1)(p)
    assert lib.sr3d_batch(arr, 1, sr3d.DATA_L1, None, None, 0, None) == -1


def test_psf_fit_host_argument_errors():
    lib = sr3d.load()
    hr, rate = sr3d.Dims(32, 32, 32), sr3d.Rate(2, 2, 2)
    rad = (ctypes.c_int * 3)(3, 3, 3)
    s0 = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    res = sr3d.PsfFitResult()

    def call(r=rad, s=s0, it=10, tol=1e-8, x=1, y=9, h=hr):
        return sr3d.STATUS[lib.sr3d_psf_fit(h, rate, x, y, ctypes.byref(r), ctypes.byref(s), it,
                                            tol, ctypes.byref(res), None, 0, None)]

    assert call() == "SR3D_ERR_WORKSPACE"
    assert call(r=(ctypes.c_int * 3)(3, -1, 3)) == "SR3D_ERR_INVALID_ARG"
    assert call(s=(ctypes.c_double * 3)(1.0, 0.0, 1.0)) == "SR3D_ERR_INVALID_ARG"
    assert call(it=0) == "SR3D_ERR_INVALID_ARG"
    assert call(tol=-1.0) == "SR3D_ERR_INVALID_ARG"
    assert call(x=None) == "SR3D_ERR_INVALID_ARG"
    assert call(h=sr3d.Dims(2, 2, 2)) == "SR3D_ERR_INVALID_ARG"  # one LR voxel
    p = sr3d.Problem()
    p.hr, p.rate = hr, rate
    assert lib.sr3d_workspace_size(sr3d.OP_PSF_FIT, ctypes.byref(p), 1) > 8 * 32 * 32 * 17


def test_multi_frame_host_argument_errors():
    lib = sr3d.load()
    hr, rate, psfd = sr3d.Dims(32, 32, 32), sr3d.Rate(2, 2, 2), sr3d.Dims(5, 5, 5)
    ptrs = (ctypes.c_void_p * 4)(1, 2, 3, 4)
    sh = (ctypes.c_int * 12)(*range(12))

    def tik(n=2, p=ptrs, s=sh, r=rate):
        return sr3d.STATUS[lib.sr3d_tikhonov_mf(hr, r, n, p, s, 9, psfd, None, 1e-3, 17, None, 0,
                                                None)]

    assert tik() == "SR3D_ERR_WORKSPACE"
    assert tik(n=0) == "SR3D_ERR_INVALID_ARG"
    assert tik(n=5) == "SR3D_ERR_INVALID_ARG"
    assert tik(s=None) == "SR3D_ERR_INVALID_ARG"
    assert tik(p=(ctypes.c_void_p * 4)(1, None, 3, 4)) == "SR3D_ERR_INVALID_ARG"
    assert tik(r=sr3d.Rate(3, 1, 1), n=1) == "SR3D_ERR_NOT_DIVISIBLE"
    p = _prob()
    assert sr3d.STATUS[lib.sr3d_tv_admm_mf(ctypes.byref(p), 2, ptrs, sh, 0, None, None, 0,
                                           None)] == "SR3D_ERR_WORKSPACE"
    for bad in (sr3d.REG_HAAR, sr3d.WARM_DUAL, sr3d.DATA_L1):
        assert lib.sr3d_tv_admm_mf(ctypes.byref(p), 2, ptrs, sh, bad, None, None, 0, None) == -1
    q = sr3d.Problem()
    q.hr, q.rate, q.psf_dims = hr, rate, psfd
    n1 = lib.sr3d_workspace_size(sr3d.OP_TIKHONOV_MF, ctypes.byref(q), 1)
    n3 = lib.sr3d_workspace_size(sr3d.OP_TIKHONOV_MF, ctypes.byref(q), 3)
    assert n3 > n1 > 0 and lib.sr3d_workspace_size(sr3d.OP_TIKHONOV_MF, ctypes.byref(q), 5) == 0
    assert lib.sr3d_workspace_size(sr3d.OP_TV_ADMM_MF, ctypes.byref(q), 2) > n3
