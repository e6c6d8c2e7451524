"""Thin ctypes binding of libsr3d (include/sr3d.h).

Argument marshalling only: tensors are torch CUDA tensors (float32, C order
(s, n, m)); their device pointers and the current stream are passed to the C
ABI, where every step of the solvers runs in HIP kernels. There is no CPU
fallback: loading fails loudly if libsr3d.so is missing.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsr3d.so")

SR3D_OK = 0
STATUS = {0: "SR3D_OK", -1: "SR3D_ERR_INVALID_ARG", -2: "SR3D_ERR_NOT_DIVISIBLE",
          -3: "SR3D_ERR_PSF_TOO_LARGE", -4: "SR3D_ERR_UNSUPPORTED_SIZE",
          -5: "SR3D_ERR_WORKSPACE", -6: "SR3D_ERR_SINGULAR", -7: "SR3D_ERR_NONFINITE",
          -8: "SR3D_ERR_HIP"}

FP64_REDUCE = 0x1
RESUME = 0x2
USE_GRAPH = 0x4
PROFILE = 0x8
WARM_DUAL = 0x10
UNFUSED = 0x20
SEPARATE_R2C = 0x40
TV_ANISO = 0x80
REG_HAAR = 0x100000
DATA_L1 = 0x200000


def HAAR_LEVELS(j):
    """Haar levels for REG_HAAR (1..8)."""
    return (j & 0xF) << 16


def CHECK_INTERVAL(k):
    return (int(k) & 0xFF) << 8


OP_TIKHONOV, OP_TV_ADMM, OP_BATCH, OP_DEGRADE, OP_FFT, OP_PSF_FIT = 1, 2, 3, 4, 5, 6
OP_TIKHONOV_MF, OP_TV_ADMM_MF = 7, 8
MAX_FRAMES = 4

EXPORTS = ["sr3d_workspace_size", "sr3d_tikhonov", "sr3d_tikhonov_noalloc", "sr3d_tv_admm", "sr3d_psf_fit",
           "sr3d_tikhonov_mf", "sr3d_tv_admm_mf", "sr3d_batch",
           "sr3d_degrade", "sr3d_rfft3d", "sr3d_irfft3d", "sr3d_cnn_param_count",
           "sr3d_cnn_init", "sr3d_cnn_workspace_size", "sr3d_cnn_forward", "sr3d_cnn_grad",
           "sr3d_cnn_adam", "sr3d_conv3d_workspace_size", "sr3d_conv3d_forward",
           "sr3d_conv3d_backward", "sr3d_autotune",
           "sr3d_tune_save", "sr3d_tune_load", "sr3d_profile_read",
           "sr3d_profile_reset", "sr3d_profile_select", "sr3d_status_string", "sr3d_last_error",
           "sr3d_shutdown"]


class Dims(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("n", ctypes.c_int), ("s", ctypes.c_int)]


class Rate(ctypes.Structure):
    _fields_ = [("dr", ctypes.c_int), ("dc", ctypes.c_int), ("ds", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("primal_rel", ctypes.c_double), ("dual_rel", ctypes.c_double),
                ("objective", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("hr", Dims), ("rate", Rate), ("y", ctypes.c_void_p), ("psf", ctypes.c_void_p),
                ("psf_dims", Dims), ("lambda_tv", ctypes.c_float), ("mu", ctypes.c_float),
                ("tol", ctypes.c_float), ("max_iter", ctypes.c_int), ("x0", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("state", ctypes.c_void_p), ("tol_dual", ctypes.c_float),
                ("mu_data", ctypes.c_float)]


class PsfFitResult(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double * 3), ("gain", ctypes.c_double),
                ("offset", ctypes.c_double), ("objective", ctypes.c_double),
                ("passes", ctypes.c_int), ("converged", ctypes.c_int)]


class Sr3dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libsr3d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} missing: run paper_2010_15491_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp, sz, ci, cf = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_float
        lib.sr3d_workspace_size.argtypes = [ci, ctypes.POINTER(Problem), ci]
        lib.sr3d_workspace_size.restype = sz
        lib.sr3d_tikhonov.argtypes = [Dims, Rate, vp, vp, Dims, vp, cf, vp, vp, sz, vp]
        lib.sr3d_tikhonov.restype = ci
        lib.sr3d_tikhonov_noalloc.argtypes = [Dims, Rate, vp, vp, Dims, vp, cf, vp, vp]
        lib.sr3d_tikhonov_noalloc.restype = ci
        lib.sr3d_psf_fit.argtypes = [Dims, Rate, vp, vp, ctypes.POINTER(ctypes.c_int * 3),
                                     ctypes.POINTER(ctypes.c_double * 3), ci, ctypes.c_double,
                                     ctypes.POINTER(PsfFitResult), vp, sz, vp]
        lib.sr3d_psf_fit.restype = ci
        lib.sr3d_tikhonov_mf.argtypes = [Dims, Rate, ci, ctypes.POINTER(vp),
                                         ctypes.POINTER(ctypes.c_int), vp, Dims, vp, cf, vp, vp,
                                         sz, vp]
        lib.sr3d_tikhonov_mf.restype = ci
        lib.sr3d_tv_admm_mf.argtypes = [ctypes.POINTER(Problem), ci, ctypes.POINTER(vp),
                                        ctypes.POINTER(ctypes.c_int), ci, ctypes.POINTER(Stats),
                                        vp, sz, vp]
        lib.sr3d_tv_admm_mf.restype = ci
        lib.sr3d_tv_admm.argtypes = [ctypes.POINTER(Problem), ci, ctypes.POINTER(Stats), vp, sz, vp]
        lib.sr3d_tv_admm.restype = ci
        lib.sr3d_batch.argtypes = [ctypes.POINTER(Problem), ci, ci, ctypes.POINTER(Stats), vp, sz, vp]
        lib.sr3d_batch.restype = ci
        lib.sr3d_degrade.argtypes = [Dims, Rate, vp, vp, Dims, vp, vp, sz, vp]
        lib.sr3d_degrade.restype = ci
        lib.sr3d_rfft3d.argtypes = [Dims, vp, vp, vp]
        lib.sr3d_rfft3d.restype = ci
        lib.sr3d_irfft3d.argtypes = [Dims, vp, vp, vp]
        lib.sr3d_irfft3d.restype = ci
        lib.sr3d_status_string.argtypes = [ci]
        lib.sr3d_status_string.restype = ctypes.c_char_p
        lib.sr3d_last_error.argtypes = []
        lib.sr3d_last_error.restype = ctypes.c_char_p
        lib.sr3d_cnn_param_count.argtypes = []
        lib.sr3d_cnn_param_count.restype = sz
        lib.sr3d_cnn_init.argtypes = [vp, ctypes.c_ulonglong, vp]
        lib.sr3d_cnn_init.restype = ci
        lib.sr3d_cnn_workspace_size.argtypes = [Dims, ci]
        lib.sr3d_cnn_workspace_size.restype = sz
        lib.sr3d_cnn_forward.argtypes = [Dims, vp, vp, vp, vp, sz, vp]
        lib.sr3d_cnn_forward.restype = ci
        lib.sr3d_cnn_grad.argtypes = [Dims, vp, vp, vp, vp, vp, vp, sz, vp]
        lib.sr3d_cnn_grad.restype = ci
        lib.sr3d_cnn_adam.argtypes = [vp, vp, vp, vp, ci, cf, cf, cf, cf, vp]
        lib.sr3d_cnn_adam.restype = ci
        lib.sr3d_conv3d_workspace_size.argtypes = [Dims]
        lib.sr3d_conv3d_workspace_size.restype = sz
        lib.sr3d_conv3d_forward.argtypes = [Dims, ci, ci, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        lib.sr3d_conv3d_forward.restype = ci
        lib.sr3d_conv3d_backward.argtypes = [Dims, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        lib.sr3d_conv3d_backward.restype = ci
        lib.sr3d_autotune.argtypes = [ctypes.POINTER(Problem), ci, ci, vp]
        lib.sr3d_autotune.restype = ci
        lib.sr3d_tune_save.argtypes = [ctypes.c_char_p]
        lib.sr3d_tune_save.restype = ci
        lib.sr3d_tune_load.argtypes = [ctypes.c_char_p]
        lib.sr3d_tune_load.restype = ci
        lib.sr3d_profile_read.argtypes = [ci, ctypes.POINTER(ctypes.c_char_p),
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_long)]
        lib.sr3d_profile_read.restype = ci
        lib.sr3d_profile_reset.argtypes = []
        lib.sr3d_profile_reset.restype = None
        lib.sr3d_profile_select.argtypes = [ctypes.c_uint]
        lib.sr3d_profile_select.restype = None
        lib.sr3d_shutdown.argtypes = []
        lib.sr3d_shutdown.restype = None
        _lib = lib
    return _lib


def _check(rc):
    if rc != SR3D_OK:
        raise Sr3dError(rc, load().sr3d_last_error().decode())


def dims_of(shape):
    """(s, n, m) array shape -> Dims(m, n, s)."""
    s, n, m = (int(v) for v in shape)
    return Dims(m, n, s)


def rate_of(rate):
    dr, dc, ds = (int(v) for v in rate)
    return Rate(dr, dc, ds)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a CUDA float32 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def workspace_bytes(op, problems):
    arr = (Problem * len(problems))(*problems)
    return int(load().sr3d_workspace_size(op, arr, len(problems)))


def workspace_bytes_n(op, problem, count):
    """sr3d_workspace_size for one problem with a count (frames of a
    multi-frame op)."""
    return int(load().sr3d_workspace_size(op, ctypes.byref(problem), int(count)))


def _workspace(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _problem(hr_shape, rate, psf, lam=1.0, mu=1.0, tol=0.0, max_iter=1, y=None, x=None, x0=None,
             state=None, tol_dual=0.0, mu_data=0.0):
    return Problem(dims_of(hr_shape), rate_of(rate), _ptr(y), _ptr(psf), dims_of(psf.shape),
                   float(lam), float(mu), float(tol), int(max_iter), _ptr(x0), _ptr(x), _ptr(state),
                   float(tol_dual), float(mu_data))


def lr_shape(hr_shape, rate):
    s, n, m = hr_shape
    dr, dc, ds = rate
    return (s // ds, n // dc, m // dr)


def hr_shape(lr, rate):
    s, n, m = lr
    dr, dc, ds = rate
    return (s * ds, n * dc, m * dr)


def tikhonov(y, psf, rate, lam, xbar=None, out=None, stream=None):
    """3D-FSR-l2-l2 (eq. (12)): returns x (HR, float32, on y's device)."""
    import torch
    _dev_f32(y, "y")
    _dev_f32(psf, "psf")
    if xbar is not None:
        _dev_f32(xbar, "xbar")
    hr = hr_shape(tuple(y.shape), rate)
    x = out if out is not None else torch.empty(hr, dtype=torch.float32, device=y.device)
    p = _problem(hr, rate, psf)
    ws = _workspace(workspace_bytes(OP_TIKHONOV, [p]), y.device)
    _check(load().sr3d_tikhonov(dims_of(hr), rate_of(rate), _ptr(y), _ptr(psf), dims_of(psf.shape),
                                _ptr(xbar), float(lam), _ptr(x), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return x


NOALLOC_SCRATCH_BYTES = 64 << 20


def tikhonov_noalloc(y, psf, rate, lam, xbar=None, out=None, stream=None):
    """eq. (12) through sr3d_tikhonov_noalloc: the library's static device
    scratch instead of a workspace (calls on one GPU must not overlap)."""
    import torch
    _dev_f32(y, "y")
    _dev_f32(psf, "psf")
    if xbar is not None:
        _dev_f32(xbar, "xbar")
    hr = hr_shape(tuple(y.shape), rate)
    x = out if out is not None else torch.empty(hr, dtype=torch.float32, device=y.device)
    _check(load().sr3d_tikhonov_noalloc(dims_of(hr), rate_of(rate), _ptr(y), _ptr(psf),
                                        dims_of(psf.shape), _ptr(xbar), float(lam), _ptr(x),
                                        _stream(stream)))
    return x


def _frames(ys, shifts):
    if len(ys) != len(shifts) or not 1 <= len(ys) <= MAX_FRAMES:
        raise ValueError(f"1..{MAX_FRAMES} frames, one shift (t_m, t_n, t_s) each")
    for y in ys:
        _dev_f32(y, "frame")
    ptrs = (ctypes.c_void_p * len(ys))(*[_ptr(y) for y in ys])
    sh = (ctypes.c_int * (3 * len(ys)))(*[int(v) for t in shifts for v in t])
    return ptrs, sh


def tikhonov_mf(ys, shifts, psf, rate, lam, xbar=None, out=None, stream=None):
    """Multi-frame Tikhonov: frames ys[f] (LR, device) observed after HR
    shifts shifts[f] = (t_m, t_n, t_s); returns x (HR)."""
    import torch
    ptrs, sh = _frames(ys, shifts)
    _dev_f32(psf, "psf")
    if xbar is not None:
        _dev_f32(xbar, "xbar")
    hr = hr_shape(tuple(ys[0].shape), rate)
    x = out if out is not None else torch.empty(hr, dtype=torch.float32, device=ys[0].device)
    p = _problem(hr, rate, psf)
    ws = _workspace(workspace_bytes_n(OP_TIKHONOV_MF, p, len(ys)), ys[0].device)
    _check(load().sr3d_tikhonov_mf(dims_of(hr), rate_of(rate), len(ys), ptrs, sh, _ptr(psf),
                                   dims_of(psf.shape), _ptr(xbar), float(lam), _ptr(x), _ptr(ws),
                                   ws.numel(), _stream(stream)))
    return x


def tv_admm_mf(ys, shifts, psf, rate, lam, mu, max_iter, tol=0.0, x0=None, flags=FP64_REDUCE,
               out=None, stream=None):
    """Algorithm 1 with the multi-frame data term. Returns (x, AdmmStats)."""
    import torch
    ptrs, sh = _frames(ys, shifts)
    _dev_f32(psf, "psf")
    if x0 is not None:
        _dev_f32(x0, "x0")
    hr = hr_shape(tuple(ys[0].shape), rate)
    x = out if out is not None else torch.empty(hr, dtype=torch.float32, device=ys[0].device)
    p = _problem(hr, rate, psf, lam, mu, tol, max_iter, y=ys[0], x=x, x0=x0)
    ws = _workspace(workspace_bytes_n(OP_TV_ADMM_MF, p, len(ys)), ys[0].device)
    st = Stats()
    _check(load().sr3d_tv_admm_mf(ctypes.byref(p), len(ys), ptrs, sh, int(flags), ctypes.byref(st),
                                  _ptr(ws), ws.numel(), _stream(stream)))
    return x, _stats(st)


def psf_fit(x, y, rate, radius, sigma0=(1.0, 1.0, 1.0), max_iter=50, tol=1e-6, stream=None):
    """Gaussian PSF estimation (sr3d_psf_fit) from an HR reference x and the
    LR volume y. radius and sigma0 are (m, n, s). Returns a dict with sigma
    (m, n, s), gain, offset, objective, passes, converged."""
    _dev_f32(x, "x")
    _dev_f32(y, "y")
    hr = tuple(x.shape)
    p = Problem()
    p.hr, p.rate = dims_of(hr), rate_of(rate)
    ws = _workspace(workspace_bytes(OP_PSF_FIT, [p]), x.device)
    res = PsfFitResult()
    rad = (ctypes.c_int * 3)(*[int(r) for r in radius])
    s0 = (ctypes.c_double * 3)(*[float(v) for v in sigma0])
    _check(load().sr3d_psf_fit(dims_of(hr), rate_of(rate), _ptr(x), _ptr(y), ctypes.byref(rad),
                               ctypes.byref(s0), int(max_iter), float(tol), ctypes.byref(res),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return {"sigma": tuple(res.sigma), "gain": res.gain, "offset": res.offset,
            "objective": res.objective, "passes": res.passes, "converged": bool(res.converged)}


@dataclass
class AdmmStats:
    iters: int
    converged: bool
    primal_rel: float
    dual_rel: float
    objective: float


def _stats(s):
    return AdmmStats(int(s.iters), bool(s.converged), float(s.primal_rel), float(s.dual_rel),
                     float(s.objective))


def tv_admm(y, psf, rate, lam, mu, max_iter, tol=0.0, x0=None, flags=FP64_REDUCE, state=None,
            out=None, workspace=None, stream=None, tol_dual=0.0, mu_data=0.0):
    """3D-FSR-l2-TV (Algorithm 1). Returns (x, AdmmStats). With DATA_L1 in
    ``flags`` the data term is ||DHx - y||_1 and ``mu_data`` the penalty of
    its split."""
    import torch
    _dev_f32(y, "y")
    _dev_f32(psf, "psf")
    if x0 is not None:
        _dev_f32(x0, "x0")
    if state is not None:
        _dev_f32(state, "state")
    hr = hr_shape(tuple(y.shape), rate)
    x = out if out is not None else torch.empty(hr, dtype=torch.float32, device=y.device)
    p = _problem(hr, rate, psf, lam, mu, tol, max_iter, y=y, x=x, x0=x0, state=state,
                 tol_dual=tol_dual, mu_data=mu_data)
    need = workspace_bytes(OP_TV_ADMM, [p])
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, y.device)
    st = Stats()
    _check(load().sr3d_tv_admm(ctypes.byref(p), int(flags), ctypes.byref(st), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return x, _stats(st)


def batch(problems, flags=FP64_REDUCE, workspace=None, stream=None):
    """Solve many TV problems. ``problems`` is a list of dicts with keys
    y, psf, rate, lam, mu, max_iter, tol, and optional x0, x. Returns
    (list of x, list of AdmmStats)."""
    import torch
    ps, xs = [], []
    for q in problems:
        y, psf = _dev_f32(q["y"], "y"), _dev_f32(q["psf"], "psf")
        hr = hr_shape(tuple(y.shape), q["rate"])
        x = q.get("x")
        if x is None:
            x = torch.empty(hr, dtype=torch.float32, device=y.device)
        xs.append(x)
        ps.append(_problem(hr, q["rate"], psf, q["lam"], q["mu"], q.get("tol", 0.0),
                           q["max_iter"], y=y, x=x, x0=q.get("x0"),
                           tol_dual=q.get("tol_dual", 0.0)))
    arr = (Problem * len(ps))(*ps)
    need = int(load().sr3d_workspace_size(OP_BATCH, arr, len(ps)))
    dev = problems[0]["y"].device
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
    sts = (Stats * len(ps))()
    _check(load().sr3d_batch(arr, len(ps), int(flags), sts, _ptr(ws), ws.numel(), _stream(stream)))
    return xs, [_stats(s) for s in sts]


def degrade(x, psf, rate, stream=None):
    """y = D H x (eq. (1) without noise)."""
    import torch
    _dev_f32(x, "x")
    _dev_f32(psf, "psf")
    hr = tuple(x.shape)
    y = torch.empty(lr_shape(hr, rate), dtype=torch.float32, device=x.device)
    p = _problem(hr, rate, psf)
    ws = _workspace(workspace_bytes(OP_DEGRADE, [p]), x.device)
    _check(load().sr3d_degrade(dims_of(hr), rate_of(rate), _ptr(x), _ptr(psf), dims_of(psf.shape),
                               _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


def rfft3d(x, stream=None):
    """Unnormalised 3D R2C DFT: returns complex64 (s, n, m//2+1)."""
    import torch
    _dev_f32(x, "x")
    s, n, m = x.shape
    spec = torch.empty((s, n, m // 2 + 1, 2), dtype=torch.float32, device=x.device)
    _check(load().sr3d_rfft3d(dims_of(x.shape), _ptr(x), _ptr(spec), _stream(stream)))
    return torch.view_as_complex(spec)


def irfft3d(spec, shape, stream=None):
    """Inverse of rfft3d (scaled by 1/N). ``spec`` is consumed (overwritten)."""
    import torch
    sp = torch.view_as_real(spec)
    if not sp.is_contiguous():
        raise ValueError("spectrum must be contiguous")
    out = torch.empty(tuple(shape), dtype=torch.float32, device=spec.device)
    _check(load().sr3d_irfft3d(dims_of(shape), _ptr(sp), _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# Learned warm start
# ---------------------------------------------------------------------------

def cnn_param_count():
    return int(load().sr3d_cnn_param_count())


def cnn_init(seed, device="cuda", stream=None):
    import torch
    p = torch.empty(cnn_param_count(), dtype=torch.float32, device=device)
    _check(load().sr3d_cnn_init(_ptr(p), int(seed), _stream(stream)))
    return p


class CnnWorkspace:
    """Reusable workspaces for one volume size."""

    def __init__(self, shape, device="cuda"):
        import torch
        self.shape = tuple(shape)
        d = dims_of(shape)
        self.fwd = torch.empty(int(load().sr3d_cnn_workspace_size(d, 0)), dtype=torch.uint8,
                               device=device)
        self.train = None
        self.device = device

    def training(self):
        import torch
        if self.train is None:
            self.train = torch.empty(int(load().sr3d_cnn_workspace_size(dims_of(self.shape), 1)),
                                     dtype=torch.uint8, device=self.device)
        return self.train


def cnn_forward(params, x, out=None, ws=None, stream=None):
    """x0 = x + f(x)."""
    import torch
    _dev_f32(params, "params")
    _dev_f32(x, "x")
    ws = ws or CnnWorkspace(x.shape, x.device)
    y = out if out is not None else torch.empty_like(x)
    _check(load().sr3d_cnn_forward(dims_of(x.shape), _ptr(params), _ptr(x), _ptr(y), _ptr(ws.fwd),
                                   ws.fwd.numel(), _stream(stream)))
    return y


def cnn_grad(params, x, target, grad=None, loss=None, ws=None, stream=None):
    """(loss, grad) of mean((x + f(x) - target)^2); loss is a 1-element tensor."""
    import torch
    _dev_f32(params, "params")
    _dev_f32(x, "x")
    _dev_f32(target, "target")
    ws = ws or CnnWorkspace(x.shape, x.device)
    g = grad if grad is not None else torch.empty_like(params)
    ls = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=x.device)
    t = ws.training()
    _check(load().sr3d_cnn_grad(dims_of(x.shape), _ptr(params), _ptr(x), _ptr(target), _ptr(g),
                                _ptr(ls), _ptr(t), t.numel(), _stream(stream)))
    return ls, g


def cnn_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().sr3d_cnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                float(beta1), float(beta2), float(eps), _stream(stream)))


def _dev_bf16(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.bfloat16:
        raise TypeError(f"{name} must be a CUDA bfloat16 tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def conv3d_forward(shape, weight, bias, x=None, act=None, stream=None):
    """One layer: 1->32 from the FP32 volume x, or 32->32 from act (bf16,
    (s, n, m, 32)). Returns (out bf16 (s, n, m, 32), out FP32 before rounding)."""
    import torch
    cin = 1 if act is None else 32
    if cin == 1:
        _dev_f32(x, "x")
    else:
        _dev_bf16(act, "act")
    dev = weight.device
    out = torch.empty(tuple(shape) + (32,), dtype=torch.bfloat16, device=dev)
    out32 = torch.empty(tuple(shape) + (32,), dtype=torch.float32, device=dev)
    d = dims_of(shape)
    ws = torch.empty(int(load().sr3d_conv3d_workspace_size(d)), dtype=torch.uint8, device=dev)
    _check(load().sr3d_conv3d_forward(d, cin, 32, _ptr(act), _ptr(x), _ptr(weight), _ptr(bias),
                                      _ptr(out), _ptr(out32), _ptr(ws), ws.numel(),
                                      _stream(stream)))
    return out, out32


def conv3d_backward(shape, act_in, gout, weight, mask=None, stream=None):
    """32->32 layer backward: returns (gweight+gbias FP32 (27*32*32+32,),
    gin bf16 or None, gin FP32 or None)."""
    import torch
    _dev_bf16(act_in, "act_in")
    _dev_bf16(gout, "gout")
    dev = weight.device
    gw = torch.empty(27 * 32 * 32 + 32, dtype=torch.float32, device=dev)
    gin = gin32 = None
    if mask is not None:
        _dev_bf16(mask, "mask")
        gin = torch.empty(tuple(shape) + (32,), dtype=torch.bfloat16, device=dev)
        gin32 = torch.empty(tuple(shape) + (32,), dtype=torch.float32, device=dev)
    d = dims_of(shape)
    ws = torch.empty(int(load().sr3d_conv3d_workspace_size(d)), dtype=torch.uint8, device=dev)
    _check(load().sr3d_conv3d_backward(d, _ptr(act_in), _ptr(gout), _ptr(weight), _ptr(mask),
                                       _ptr(gin), _ptr(gin32), _ptr(gw), _ptr(ws), ws.numel(),
                                       _stream(stream)))
    return gw, gin, gin32


def autotune(shapes_rates, force=False, stream=None):
    """Tune the FFT tile variants for HR shapes (s, n, m) with their rates
    [(shape, rate), ...] (and the LR sizes they imply)."""
    ps = []
    for shape, rate in shapes_rates:
        p = Problem()
        p.hr, p.rate, p.psf_dims = dims_of(shape), rate_of(rate), Dims(1, 1, 1)
        ps.append(p)
    arr = (Problem * len(ps))(*ps)
    _check(load().sr3d_autotune(arr, len(ps), int(bool(force)), _stream(stream)))


def tune_save(path):
    _check(load().sr3d_tune_save(str(path).encode()))


def tune_load(path):
    rc = load().sr3d_tune_load(str(path).encode())
    if rc < 0:
        _check(rc)
    return rc


def profile_reset():
    load().sr3d_profile_reset()


def profile_read():
    """{stage name: (total_ms, launches)} gathered by calls made with PROFILE."""
    lib = load()
    out = {}
    i = 0
    while True:
        name, ms, n = ctypes.c_char_p(), ctypes.c_double(), ctypes.c_long()
        if lib.sr3d_profile_read(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(n)) != 0:
            break
        out[name.value.decode()] = (ms.value, n.value)
        i += 1
    return out


def profile_select(stages=None):
    """Time only the named stages under PROFILE (None: every stage)."""
    lib = load()
    if stages is None:
        mask = 0xFFFFFFFF
    else:
        names, i = {}, 0
        while True:
            name = ctypes.c_char_p()
            if lib.sr3d_profile_read(i, ctypes.byref(name), None, None) != 0:
                break
            names[name.value.decode()] = i
            i += 1
        mask = 0
        for st in stages:
            mask |= 1 << names[st]
    lib.sr3d_profile_select(ctypes.c_uint(mask))


def shutdown():
    load().sr3d_shutdown()
