#!/usr/bin/env python3
"""Benchmark of the Fourier-domain TV-ADMM super-resolution solver on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one complete TV-ADMM solve (Algorithm 1 of Tuador et al.) of a
256^3 HR volume from a 128^3 LR volume (d = 2x2x2, Gaussian PSF sigma 1.5,
7^3 taps, lambda_TV 2e-3, mu 5e-2, relative residual tolerance 1e-4, cap 200
iterations): setup (PSF spectrum, LR spectrum, symbol tables), every x-update
(3D R2C FFT, fold/solve/unfold, 3D C2R FFT), every difference/shrink/dual
step and every residual reduction and stopping test, from device-resident y
to device-resident x. Inputs are a seeded synthetic ellipsoid phantom with a
smooth texture field, blurred and decimated on the GPU, plus seeded noise.

Prints one JSON line: HR voxels per second, the per-kernel roofline of the
dominant kernel (HIP-event durations measured inside the timed steps) and the
FP64 CPU oracle timed on a bounded sample on this host.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HR voxels/s, TV-ADMM 256³ d=2³ to 1e-4 tol; % HBM peak; vs plain/warm"
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(name="tv_admm_256cube_d2x2x2_tol1e-4_cap200", hr=(256, 256, 256),
                rate=(2, 2, 2), sigma=1.5, noise=0.02, lam=2e-3, mu=5e-2, tol=1e-4,
                max_iter=200, seed=1, texture=True)


def alg_bytes_per_voxel(stage, hr, rate):
    """Algorithmic HBM bytes per HR voxel for one launch of a stage: every array
    the stage must read or write, counted once, at its stored size."""
    S, N, M = hr
    dr, dc, ds = rate
    mh = (M // 2 + 1) / M          # half-spectrum columns per real column
    ml = M // dr
    mlh = (ml // 2 + 1) / ml
    d = dr * dc * ds
    spec = 8.0 * mh                # complex64 half spectrum per HR voxel
    table = {
        "fft_r2c_m": 4.0 + spec,
        "fft_c2c_n": 2 * spec, "fft_c2c_s": 2 * spec,
        "ifft_c2c_s": 2 * spec, "ifft_c2c_n": 2 * spec,
        "ifft_c2r_m": spec + 4.0,
        # F Theta, Lambda, LR spectrum of y (per HR voxel: 1/d of an LR entry), X
        "fold_solve": 3 * spec + 8.0 * mlh / d,
        # fused s-FFT + solve + inverse s-FFT: the spectrum read and written
        # once, Lambda and the LR spectrum of y read once
        "solve_s": 3 * spec + 8.0 * mlh / d,
        # x and nu_old (3 planes) read; nu_new (3 planes) and Theta written
        "admm_stencil": 4.0 + 12.0 + 12.0 + 4.0,
        # the same with the m-axis R2C fused in: Theta's half spectrum written
        "stencil_r2c": 4.0 + 12.0 + 12.0 + spec,
        # Haar form, steps 5b/5c and W, W^T: x and nu_old read, nu_new and
        # xbar written (one plane each)
        "wavelet": 4.0 + 4.0 + 4.0 + 4.0,
    }
    return table.get(stage)


def kernel_source_sha(path):
    """SHA-256 (16 hex digits) over a kernel's source file and, transitively,
    the local headers it includes (`#include "name"` in the same folder)."""
    h, seen, todo = hashlib.sha256(), set(), [path]
    while todo:
        rel = todo.pop(0)
        if rel in seen:
            continue
        seen.add(rel)
        with open(os.path.join(ROOT, rel), "rb") as f:
            text = f.read()
        h.update(rel.encode() + b"\0" + text)
        folder = os.path.dirname(rel)
        for m in re.finditer(rb'^\s*#\s*include\s+"([^"]+)"', text, re.M):
            inc = os.path.join(folder, m.group(1).decode())
            if os.path.exists(os.path.join(ROOT, inc)):
                todo.append(inc)
    return h.hexdigest()[:16]


def traffic_for(stage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current source of the stage's kernel; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(stage)
    if not rec:
        return None
    if kernel_source_sha(rec["source"]) != rec["source_sha"]:
        return None
    return rec["bytes_per_launch"]


def make_inputs(torch, sr3d, phantom, wl, dev):
    p = phantom.make_problem(wl["hr"], wl["rate"], wl["sigma"], wl["noise"], wl["seed"],
                             texture=wl["texture"])
    psf = torch.from_numpy(p["psf"].astype("float32")).to(dev)
    x_true = torch.from_numpy(p["x_true"].astype("float32")).to(dev)
    y = sr3d.degrade(x_true, psf, wl["rate"])
    y += torch.from_numpy(p["noise"].astype("float32")).to(dev)
    torch.cuda.synchronize()
    return y.contiguous(), psf, x_true


def host_cpu_model():
    """The host CPU's model name (first `model name` line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(y_np, psf_np, wl, iters_gpu, iters_timed=10):
    """FP64 oracle on this host, on the same inputs: Algorithm 1 with 1 and
    1 + iters_timed iterations (all of this process's cores for the FFTs),
    giving seconds per iteration and the setup; the rate is setup + the GPU
    run's iteration count. The same with one FFT worker, 1 and 3 iterations,
    gives the single-thread figure."""
    import oracle as O

    def per_iter(k):
        t0 = time.perf_counter()
        O.admm_tv(y_np, psf_np, wl["rate"], wl["lam"], wl["mu"], 1)
        t1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.admm_tv(y_np, psf_np, wl["rate"], wl["lam"], wl["mu"], 1 + k)
        tk = time.perf_counter() - t0
        it = max((tk - t1) / k, 1e-9)
        return it, max(t1 - it, 0.0), t1, tk

    cores = int(O.WORKERS)
    it_all, setup_all, t1, tk = per_iter(iters_timed)
    saved = O.WORKERS
    try:
        O.WORKERS = 1
        it_one, setup_one, t1s, tks = per_iter(2)
    finally:
        O.WORKERS = saved
    nh = wl["hr"][0] * wl["hr"][1] * wl["hr"][2]
    total = setup_all + iters_gpu * it_all
    return {"value": nh / total, "unit": "HR voxels/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 oracle admm_tv on the same 256^3 inputs with {cores} FFT threads: "
                       f"1 and {1 + iters_timed} iterations timed ({t1:.1f} s, {tk:.1f} s); "
                       f"setup {setup_all:.2f} s + {iters_gpu} x {it_all:.2f} s/iteration, "
                       "scaled to the GPU run's iteration count"),
            "seconds_per_iteration": it_all, "setup_seconds": setup_all,
            "iterations_timed": 1 + iters_timed,
            "single_thread": {"seconds_per_iteration": it_one, "setup_seconds": setup_one,
                              "value": nh / (setup_one + iters_gpu * it_one),
                              "sample": f"1 and 3 iterations with 1 FFT thread ({t1s:.1f} s, "
                                        f"{tks:.1f} s)"},
            "host_nproc": os.cpu_count(), "host_cpu_model": host_cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="tv256: skip the batched and warm-started forms measured after the "
                         "timed steps (the 'forms' record)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps without per-kernel HIP events (no roofline)")
    ap.add_argument("--workload", default="tv256",
                    choices=["tv256", "batch64", "warm256", "psf256", "mf256", "cnn256"],
                    help="tv256: the headline single-volume solve; batch64: 64 uneven volumes, "
                         "sequential single solves vs one batched solve; warm256: train the "
                         "warm-start CNN on 64^3 pairs, then plain vs warm-started solves at 256^3; "
                         "psf256: Gaussian PSF fit from a 256^3 reference and its 128^3 LR volume; "
                         "mf256: multi-frame TV-ADMM, four 128^3 frames of HR-shifted copies; "
                         "cnn256: warm-start CNN inference on a 256^3 volume (seeded random "
                         "weights) and one 64^3 training gradient per step")
    ap.add_argument("--separate-r2c", action="store_true",
                    help="tv256: run the tiled stencil and the m-axis R2C as separate kernels "
                         "(SR3D_SEPARATE_R2C) instead of the fused stencil")
    ap.add_argument("--aniso", action="store_true",
                    help="tv256: anisotropic TV (SR3D_TV_ANISO) instead of the isotropic default")
    ap.add_argument("--haar", type=int, default=0, metavar="LEVELS",
                    help="tv256: l1 of orthonormal Haar details with LEVELS levels "
                         "(SR3D_REG_HAAR) instead of TV")
    ap.add_argument("--data-l1", type=float, default=0.0, metavar="MU_DATA",
                    help="tv256: l1 data term (SR3D_DATA_L1) with this data-split penalty, on the "
                         "same volume with impulses (+-1 on 10%% of the LR voxels) added to y")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the timed steps, copy a buffer of this many MiB once (a dispatch "
                         "of known traffic for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--batch-only", action="store_true",
                    help="batch64: time the batched solve alone, without the sequential comparison "
                         "(for profiling the batch kernels)")
    ap.add_argument("--pairs", type=int, default=2000, help="warm256: training pairs")
    ap.add_argument("--train-steps", type=int, default=4000, help="warm256: Adam steps")
    ap.add_argument("--eval-volumes", type=int, default=4, help="warm256: 256^3 test volumes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the workload is one volume; see the sharding design notes)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        return bench_batch64(args)
    if args.workload == "warm256":
        return bench_warm256(args)
    if args.workload == "psf256":
        return bench_psf256(args)
    if args.workload == "mf256":
        return bench_mf256(args)
    if args.workload == "cnn256":
        return bench_cnn256(args)

    import numpy as np
    import torch
    from paper_2010_15491_amd import phantom, sr3d

    sr3d.load()
    dev = torch.device("cuda:0")
    wl = WORKLOAD
    y, psf, _ = make_inputs(torch, sr3d, phantom, wl, dev)
    if args.data_l1 > 0:
        y += torch.from_numpy(phantom.impulse_noise(tuple(y.shape), wl["seed"] + 500, 0.1, 1.0)
                              .astype("float32")).to(dev)
    hr = wl["hr"]
    nh = hr[0] * hr[1] * hr[2]
    x = torch.empty(hr, dtype=torch.float32, device=dev)
    p = sr3d._problem(hr, wl["rate"], psf, wl["lam"], wl["mu"], wl["tol"], wl["max_iter"], y=y,
                      x=x)
    ws = torch.empty(sr3d.workspace_bytes(sr3d.OP_TV_ADMM, [p]), dtype=torch.uint8, device=dev)
    base_flags = (sr3d.FP64_REDUCE | (sr3d.SEPARATE_R2C if args.separate_r2c else 0)
                  | (sr3d.TV_ANISO if args.aniso else 0)
                  | (sr3d.REG_HAAR | sr3d.HAAR_LEVELS(args.haar) if args.haar else 0)
                  | (sr3d.DATA_L1 if args.data_l1 > 0 else 0))
    flags = base_flags | (0 if args.no_profile else sr3d.PROFILE)
    flags_all = flags
    # FFT tile variants: timed once on this device, outside the timed steps.
    sr3d.autotune([(hr, wl["rate"])])
    with tempfile.TemporaryDirectory() as td:
        tune_path = os.path.join(td, "fft_tiles.txt")
        sr3d.tune_save(tune_path)
        with open(tune_path) as f:
            fft_tiles = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]

    def step(fl=None):
        return sr3d.tv_admm(y, psf, wl["rate"], wl["lam"], wl["mu"], wl["max_iter"],
                            tol=wl["tol"], flags=flags if fl is None else fl, out=x, workspace=ws,
                            mu_data=args.data_l1)

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(base_flags)
    # Per-kernel breakdown: one untimed step with every stage timed. The timed
    # steps then carry events around the dominant kernel only (each timed
    # launch adds two event records to the stream).
    kernels = {}
    dom = None
    if not args.no_profile:
        sr3d.profile_select(None)
        sr3d.profile_reset()
        _, st_b = step(flags_all)
        torch.cuda.synchronize()
        for name, (tot, n) in sr3d.profile_read().items():
            if n:
                kernels[name] = {"avg_us": 1e3 * tot / n, "launches": n, "total_ms": tot}
        iter_k = {k: v for k, v in kernels.items() if alg_bytes_per_voxel(k, hr, wl["rate"])}
        dom = max(iter_k, key=lambda k: iter_k[k]["total_ms"])
        for k, v in iter_k.items():
            b = alg_bytes_per_voxel(k, hr, wl["rate"]) * nh
            v["achieved_GBs"] = round(b / (v["avg_us"] * 1e-6) / 1e9, 1)
        kernels["_note"] = ("one untimed step with HIP events around every launch "
                            f"({st_b.iters} iterations); the timed steps time {dom} only")
        sr3d.profile_select([dom])
    sr3d.profile_reset()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    stats = None
    for _ in range(args.steps):
        _, stats = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = nh / (ms / 1e3)

    roofline = None
    if not args.no_profile:
        tot, n = sr3d.profile_read()[dom]
        avg_us = 1e3 * tot / max(n, 1)
        bpl = alg_bytes_per_voxel(dom, hr, wl["rate"]) * nh
        achieved = bpl / (avg_us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic_for(dom), "kernel": dom,
                    "alg_bytes_per_launch": int(bpl), "avg_launch_us": round(avg_us, 2),
                    "launches_timed": n, "iteration_us": round(1e3 * ms / max(stats.iters, 1), 1)}
        sr3d.profile_select(None)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(y.double().cpu().numpy(), psf.double().cpu().numpy(), wl, stats.iters)

    # The forms, each against the plain GPU method on this GPU, measured after
    # the timed steps (not part of `value`).
    forms = None
    if not (args.no_forms or args.separate_r2c or args.aniso or args.haar or args.data_l1 > 0):
        del ws
        torch.cuda.empty_cache()
        b = bench_batch64(argparse.Namespace(steps=1, batch_only=False), emit=False)
        torch.cuda.empty_cache()
        w = bench_warm256(argparse.Namespace(pairs=args.pairs, train_steps=args.train_steps,
                                             eval_volumes=args.eval_volumes), emit=False)
        forms = {
            "batch64": {"volumes": b["config"]["volumes"],
                        "total_hr_voxels": b["config"]["total_hr_voxels"],
                        "sequential_ms": b["sequential"]["ms_per_step"],
                        "batched_ms": b["ms_per_step"],
                        "speedup_vs_sequential": b["speedup_vs_sequential"],
                        "same_iters_as_sequential": b["config"]["same_iters_as_sequential"],
                        "max_rel_l2_vs_sequential": b["config"]["max_rel_l2_vs_sequential"]},
            "warm256": {"volumes": len(w["runs"]), "target": "the plain solve's final residuals",
                        "plain_ms": 1e3 * w["mean_s"]["plain"],
                        "warm_ms": 1e3 * w["mean_s"]["cnn_x0"],
                        "speedup_vs_plain": w["value"],
                        "mean_iters_plain": w["mean_iters"]["plain"],
                        "mean_iters_warm": w["mean_iters"]["cnn_x0"],
                        "fallbacks": w["fallbacks"],
                        "inference_ms": 1e3 * w["cnn_inference_256"]["s"],
                        "inference_tflops": w["cnn_inference_256"]["tflops"],
                        "train_s": w["config"]["train_s"]},
        }

    out = {
        "metric": METRIC, "value": value, "unit": "HR voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "hr": list(hr), "rate": list(wl["rate"]),
                   "psf_sigma": wl["sigma"], "psf_taps": 7, "noise_sigma": wl["noise"],
                   "lambda_tv": wl["lam"], "mu": wl["mu"], "tol": wl["tol"],
                   "max_iter": wl["max_iter"], "iters": stats.iters,
                   "converged": stats.converged, "primal_rel": stats.primal_rel,
                   "dual_rel": stats.dual_rel, "reductions": "fp64",
                   "stencil": ("tiled + separate R2C" if args.separate_r2c or args.data_l1 > 0
                               else "fused R2C"),
                   "regulariser": (f"l1 of {args.haar}-level Haar details" if args.haar
                                   else "anisotropic TV" if args.aniso else "isotropic TV"),
                   "data_term": (f"l1 (mu_data {args.data_l1}, impulses on 10% of y)"
                                 if args.data_l1 > 0 else "l2"),
                   "fft_tiles_kind_len_variant": fft_tiles,
                   "parallelism": "single_gpu"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": forms,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


BATCH_SHAPES = [(64, 64, 64), (64, 96, 96), (128, 128, 128), (96, 192, 192)]  # (s, n, m)
BATCH_RATES = [(2, 2, 2), (2, 2, 4), (4, 4, 2)]                               # (dr, dc, ds)


def batch64_problems(torch, sr3d, phantom, dev, count=64, seed0=100):
    """64 volumes: shape, rate and sigma ~ U[0.8, 2.0] drawn per volume from
    numpy.random.default_rng(seed), then the phantom with the same seed."""
    import numpy as np
    probs = []
    for i in range(count):
        seed = seed0 + i
        meta = np.random.default_rng(seed)
        shape = BATCH_SHAPES[int(meta.integers(len(BATCH_SHAPES)))]
        rate = BATCH_RATES[int(meta.integers(len(BATCH_RATES)))]
        sigma = float(meta.uniform(0.8, 2.0))
        p = phantom.make_problem(shape, rate, sigma, 0.02, seed)
        psf = torch.from_numpy(p["psf"].astype("float32")).to(dev)
        xt = torch.from_numpy(p["x_true"].astype("float32")).to(dev)
        y = sr3d.degrade(xt, psf, rate)
        y += torch.from_numpy(p["noise"].astype("float32")).to(dev)
        del xt
        probs.append(dict(y=y.contiguous(), psf=psf, rate=rate, lam=2e-3, mu=5e-2, tol=1e-4,
                          max_iter=200, shape=shape, sigma=sigma,
                          x=torch.empty(shape, dtype=torch.float32, device=dev)))
    torch.cuda.synchronize()
    return probs


def bench_batch64(args, emit=True):
    """Batched form: 64 uneven volumes solved (a) one after another with the
    plain single-volume solver and (b) together by sr3d_batch (HIP-graph
    replay), to the same tolerance; reports both rates and the speedup."""
    import numpy as np
    import torch
    from paper_2010_15491_amd import phantom, sr3d

    sr3d.load()
    dev = torch.device("cuda:0")
    probs = batch64_problems(torch, sr3d, phantom, dev)
    sr3d.autotune(sorted({(q["shape"], q["rate"]) for q in probs}))
    nh = sum(int(np.prod(q["shape"])) for q in probs)
    ws_single = torch.empty(max(sr3d.workspace_bytes(sr3d.OP_TV_ADMM, [sr3d._problem(
        q["shape"], q["rate"], q["psf"], y=q["y"], x=q["x"])]) for q in probs),
        dtype=torch.uint8, device=dev)
    flags = sr3d.FP64_REDUCE

    def sequential():
        out = []
        for q in probs:
            _, st = sr3d.tv_admm(q["y"], q["psf"], q["rate"], q["lam"], q["mu"], q["max_iter"],
                                 tol=q["tol"], flags=flags, out=q["x"], workspace=ws_single)
            out.append(st)
        return out

    bflags = flags | sr3d.USE_GRAPH | sr3d.CHECK_INTERVAL(8)
    bps = [sr3d._problem(q["shape"], q["rate"], q["psf"], q["lam"], q["mu"], q["tol"],
                         q["max_iter"], y=q["y"], x=q["x"]) for q in probs]
    ws_batch = torch.empty(sr3d.workspace_bytes(sr3d.OP_BATCH, bps), dtype=torch.uint8, device=dev)

    def batched():
        _, sts = sr3d.batch(probs, flags=bflags, workspace=ws_batch)
        return sts

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            res = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, res

    reps = max(1, args.steps)
    same_iters = max_rel = ms_seq = None
    if not args.batch_only:
        ms_seq, st_seq = timed(sequential, reps)
        x_seq = [q["x"].clone() for q in probs]
    ms_bat, st_bat = timed(batched, reps)
    if ms_seq is not None:
        same_iters = sum(a.iters == b.iters for a, b in zip(st_seq, st_bat))
        max_rel = max(float(torch.linalg.vector_norm(q["x"] - xs) / torch.linalg.vector_norm(xs))
                      for q, xs in zip(probs, x_seq))
    out = {
        "metric": "HR voxels/s, 64 uneven TV-ADMM volumes to 1e-4 tol (batched vs sequential)",
        "value": nh / (ms_bat / 1e3), "unit": "HR voxels/s", "n_gpus": 1, "steps": reps,
        "warmup": 1, "ms_per_step": ms_bat, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64_uneven_tv_admm", "volumes": len(probs),
                   "total_hr_voxels": nh, "shapes_snm": BATCH_SHAPES, "rates": BATCH_RATES,
                   "iters_min": min(s.iters for s in st_bat),
                   "iters_max": max(s.iters for s in st_bat),
                   "converged": sum(s.converged for s in st_bat),
                   "same_iters_as_sequential": same_iters, "max_rel_l2_vs_sequential": max_rel},
        "sequential": (None if ms_seq is None else
                       {"value": nh / (ms_seq / 1e3), "ms_per_step": ms_seq}),
        "speedup_vs_sequential": None if ms_seq is None else ms_seq / ms_bat,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


PSF_WORKLOAD = dict(hr=(256, 256, 256), rate=(2, 2, 2), sigma=(1.8, 1.5, 1.1), radius=(6, 6, 6),
                    gain=0.9, offset=0.05, noise=0.01, seed=1)


def bench_cnn256(args):
    """Warm-start CNN alone: one step = one inference x0 = x + f(x) on a 256^3
    volume (standard normal input, network initialised from seed 7), then one
    loss gradient on a 64^3 volume. Inference FLOPs count the useful
    multiply-adds of the six layers (27 taps; 1->32, 4 x 32->32, 32->1)."""
    import torch
    from paper_2010_15491_amd import sr3d

    sr3d.load()
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(7)
    params = sr3d.cnn_init(7)
    x = torch.randn((256, 256, 256), device=dev, generator=g)
    ws = sr3d.CnnWorkspace(x.shape)
    y = sr3d.cnn_forward(params, x, ws=ws)
    x64 = torch.randn((64, 64, 64), device=dev, generator=g)
    t64 = x64 + 0.01
    ws64 = sr3d.CnnWorkspace(x64.shape)
    for _ in range(max(args.warmup, 1)):
        sr3d.cnn_forward(params, x, out=y, ws=ws)
        sr3d.cnn_grad(params, x64, t64, ws=ws64)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_inf = t_grad = 0.0
    for _ in range(args.steps):
        ev[0].record()
        sr3d.cnn_forward(params, x, out=y, ws=ws)
        ev[1].record()
        sr3d.cnn_grad(params, x64, t64, ws=ws64)
        ev[2].record()
        torch.cuda.synchronize()
        t_inf += ev[0].elapsed_time(ev[1])
        t_grad += ev[1].elapsed_time(ev[2])
    ms_inf, ms_grad = t_inf / args.steps, t_grad / args.steps
    flops = 2.0 * 256 ** 3 * 27 * (32 + 4 * 32 * 32 + 32)
    out = {"metric": "warm-start CNN inference, 256^3", "value": flops / (ms_inf / 1e3) / 1e12,
           "unit": "TFLOP/s (bf16 MFMA, useful FLOPs)", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_inf + ms_grad, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "cnn256", "inference_ms": ms_inf, "grad64_ms": ms_grad,
                      "frac_of_bf16_peak": flops / (ms_inf / 1e3) / 2.5e15}}
    print(json.dumps(out), flush=True)
    return out


def bench_psf256(args):
    """PSF estimation: the headline phantom (with texture) as the HR
    reference, y = gain D H_sigma x + offset + noise made on the GPU by the
    library's own forward model with the sampled Gaussian; the fit starts
    from sigma = 1. One step = sr3d_psf_fit including its two R2C FFTs."""
    import numpy as np
    import torch
    from paper_2010_15491_amd import phantom, sr3d

    sr3d.load()
    dev = torch.device("cuda:0")
    wl = PSF_WORKLOAD
    p = phantom.make_problem(wl["hr"], wl["rate"], 1.0, wl["noise"], wl["seed"], texture=True)
    x = torch.from_numpy(p["x_true"].astype("float32")).to(dev)
    # the fitted family: separable sampled Gaussian on 2 radius + 1 taps per axis
    taps = []
    for sg, r in zip(wl["sigma"], wl["radius"]):
        i = np.arange(-r, r + 1, dtype=np.float64)
        g = np.exp(-i * i / (2.0 * sg * sg))
        taps.append(g / g.sum())
    k3 = taps[2][:, None, None] * taps[1][None, :, None] * taps[0][None, None, :]
    psf = torch.from_numpy(k3.astype("float32")).to(dev)
    y = wl["gain"] * sr3d.degrade(x, psf, wl["rate"]) + wl["offset"]
    y += torch.from_numpy(p["noise"].astype("float32")).to(dev)
    torch.cuda.synchronize()
    for _ in range(max(args.warmup, 1)):
        res = sr3d.psf_fit(x, y, wl["rate"], wl["radius"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        res = sr3d.psf_fit(x, y, wl["rate"], wl["radius"])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nh = int(np.prod(wl["hr"]))
    out = {"metric": "HR voxels/s, Gaussian PSF fit 256^3 -> 128^3 (sigma, gain, offset)",
           "value": nh / (ms / 1e3), "unit": "HR voxels/s", "n_gpus": 1, "steps": args.steps,
           "ms_per_step": ms, "higher_is_better": True, "dtype": "f32 data, f64 sums",
           "data": "synthetic", "config": {"workload": "psf256", **{k: v for k, v in wl.items()}},
           "fit": res,
           "sigma_rel_error": [abs(a - b) / b for a, b in zip(res["sigma"], wl["sigma"])]}
    print(json.dumps(out), flush=True)


MF_WORKLOAD = dict(hr=(256, 256, 256), rate=(2, 2, 2), sigma=1.5, noise=0.02, lam=2e-3, mu=5e-2,
                   shifts=[(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)], iters=50, seed=1)


def bench_mf256(args):
    """Multi-frame TV-ADMM: four 128^3 frames of HR-shifted copies of the
    headline phantom (shifts inside the 2x2x2 block), 50 iterations."""
    import numpy as np
    import torch
    from paper_2010_15491_amd import phantom, sr3d

    sr3d.load()
    dev = torch.device("cuda:0")
    wl = MF_WORKLOAD
    p = phantom.make_problem(wl["hr"], wl["rate"], wl["sigma"], wl["noise"], wl["seed"],
                             texture=True)
    x = torch.from_numpy(p["x_true"].astype("float32")).to(dev)
    psf = torch.from_numpy(p["psf"].astype("float32")).to(dev)
    rng = np.random.default_rng(wl["seed"] + 900)
    ys = []
    for t in wl["shifts"]:
        xs = torch.roll(x, shifts=(-t[2], -t[1], -t[0]), dims=(0, 1, 2))
        y = sr3d.degrade(xs, psf, wl["rate"])
        y += torch.from_numpy((wl["noise"] * rng.standard_normal(tuple(y.shape)))
                              .astype("float32")).to(dev)
        ys.append(y)
    del x
    sr3d.autotune([(wl["hr"], wl["rate"])])

    def step():
        return sr3d.tv_admm_mf(ys, wl["shifts"], psf, wl["rate"], wl["lam"], wl["mu"], wl["iters"])

    for _ in range(max(args.warmup, 1)):
        step()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        _, st = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nh = int(np.prod(wl["hr"]))
    out = {"metric": "HR voxels/s, multi-frame TV-ADMM 256^3 from 4 frames, 50 iterations",
           "value": nh / (ms / 1e3), "unit": "HR voxels/s", "n_gpus": 1, "steps": args.steps,
           "ms_per_step": ms, "higher_is_better": True, "dtype": "f32 (f64 per-group solve)",
           "data": "synthetic", "config": {"workload": "mf256", **wl},
           "iters": st.iters, "primal_rel": st.primal_rel, "dual_rel": st.dual_rel}
    print(json.dumps(out), flush=True)


VARIANTS = ("plain", "tikhonov_x0", "cnn_x0", "tikhonov_x0_dual", "cnn_x0_dual")


def bench_warm256(args, emit=True):
    """Learned warm start: pairs from 64^3 phantoms (batched plain ADMM), GPU
    training, then on 256^3 volumes like the headline workload: iterations and
    wall time to reach the plain run's final residuals from x0 = 0, from the
    Tikhonov solution, and from the CNN (Tikhonov and inference included)."""
    import numpy as np
    import torch
    from paper_2010_15491_amd import phantom, sr3d, warmstart

    sr3d.load()
    dev = torch.device("cuda:0")
    wl = WORKLOAD
    sr3d.autotune([((64, 64, 64), (2, 2, 2)), (wl["hr"], wl["rate"])])
    (pairs, pst), t_pairs = warmstart.timed(
        lambda: warmstart.make_pairs(range(1000, 1000 + args.pairs)))
    print(f"pairs: {len(pairs)} in {t_pairs:.1f} s", file=sys.stderr, flush=True)
    (params, losses, _), t_train = warmstart.timed(
        lambda: warmstart.train(pairs, args.train_steps))
    print(f"trained {args.train_steps} steps in {t_train:.1f} s, loss {losses[0]:.3e} -> "
          f"{np.mean(losses[-50:]):.3e}", file=sys.stderr, flush=True)
    del pairs
    torch.cuda.empty_cache()
    hr, rate = wl["hr"], wl["rate"]
    nh = hr[0] * hr[1] * hr[2]
    cws = sr3d.CnnWorkspace(hr)
    x = torch.empty(hr, dtype=torch.float32, device=dev)
    ws = torch.empty(sr3d.workspace_bytes(sr3d.OP_TV_ADMM, [sr3d._problem(hr, rate, torch.ones(
        7, 7, 7, device=dev))]), dtype=torch.uint8, device=dev)
    runs = []
    for k in range(args.eval_volumes):
        p = phantom.make_problem(hr, rate, wl["sigma"], wl["noise"], 5000 + k, texture=True)
        psf = torch.from_numpy(p["psf"].astype("float32")).to(dev)
        y = sr3d.degrade(torch.from_numpy(p["x_true"].astype("float32")).to(dev), psf, rate)
        y += torch.from_numpy(p["noise"].astype("float32")).to(dev)

        def admm(x0, tol, told, dual=False):
            fl = sr3d.FP64_REDUCE | (sr3d.WARM_DUAL if dual else 0)
            return sr3d.tv_admm(y, psf, rate, wl["lam"], wl["mu"], wl["max_iter"], tol=tol,
                                tol_dual=told, x0=x0, out=x, workspace=ws, flags=fl)

        if k == 0:  # warm-up of every kernel involved
            admm(None, wl["tol"], 0.0)
            warmstart.warm_start(params, y, psf, rate, ws=cws)
        (_, st0), t0 = warmstart.timed(lambda: admm(None, wl["tol"], 0.0))
        tp, td = max(wl["tol"], st0.primal_rel), max(wl["tol"], st0.dual_rel)
        (_, stp), tpl = warmstart.timed(lambda: admm(None, tp, td))
        (_, stt), tt = warmstart.timed(
            lambda: admm(sr3d.tikhonov(y, psf, rate, 1e-3), tp, td))
        xt = sr3d.tikhonov(y, psf, rate, 1e-3)
        _, t_inf = warmstart.timed(lambda: sr3d.cnn_forward(params, xt, ws=cws))
        # the accept-or-fall-back solve: Tikhonov, inference, the warm-started
        # ADMM and, if it misses the target, plain ADMM; all of it timed
        (_, wsol), tc = warmstart.timed(
            lambda: warmstart.solve(params, y, psf, rate, wl["lam"], wl["mu"], wl["max_iter"],
                                    tol=tp, tol_dual=td, out=x, workspace=ws, cnn_ws=cws))
        stc = wsol.warm
        (_, sttd), ttd = warmstart.timed(
            lambda: admm(sr3d.tikhonov(y, psf, rate, 1e-3), tp, td, dual=True))
        (_, stcd), tcd = warmstart.timed(
            lambda: admm(warmstart.warm_start(params, y, psf, rate, ws=cws), tp, td, dual=True))
        runs.append({"seed": 5000 + k, "plain_cap_run": {"iters": st0.iters, "s": t0,
                                                         "primal": st0.primal_rel,
                                                         "dual": st0.dual_rel},
                     "target": [tp, td],
                     "plain": {"iters": stp.iters, "reached": stp.converged, "s": tpl},
                     "tikhonov_x0": {"iters": stt.iters, "reached": stt.converged, "s": tt},
                     "cnn_x0": {"iters": stc.iters, "reached": stc.converged, "s": tc,
                                "inference_s": t_inf, "used": wsol.used,
                                "fallback_iters": None if wsol.plain is None else wsol.plain.iters},
                     "tikhonov_x0_dual": {"iters": sttd.iters, "reached": sttd.converged, "s": ttd},
                     "cnn_x0_dual": {"iters": stcd.iters, "reached": stcd.converged, "s": tcd}})
        print(json.dumps(runs[-1]), file=sys.stderr, flush=True)
    flops = 2.0 * 27 * (32 + 4 * 32 * 32 + 32) * nh
    mean = lambda key, f: float(np.mean([f(r[key]) for r in runs]))
    out = {
        "metric": "warm start: wall time to the plain solve's final residuals, 256^3 TV-ADMM",
        "value": mean("plain", lambda r: r["s"]) / mean("cnn_x0", lambda r: r["s"]),
        "unit": "speedup (plain / CNN warm start; Tikhonov, inference and any fallback included)",
        "fallbacks": int(sum(r["cnn_x0"]["used"] == "plain" for r in runs)),
        "n_gpus": 1,
        "higher_is_better": True, "dtype": "f32 solver, bf16 CNN", "data": "synthetic",
        "config": {"workload": "warm256", "train_pairs": args.pairs, "train_steps": args.train_steps,
                   "pair_generation_s": t_pairs, "train_s": t_train,
                   "train_loss_first": losses[0], "train_loss_last50": float(np.mean(losses[-50:])),
                   "pair_admm_converged": int(sum(s.converged for s in pst))},
        "cnn_inference_256": {"s": float(np.mean([r["cnn_x0"]["inference_s"] for r in runs])),
                              "tflops": flops / float(np.mean([r["cnn_x0"]["inference_s"]
                                                               for r in runs])) / 1e12},
        "mean_iters": {k: mean(k, lambda r: r["iters"]) for k in VARIANTS},
        "mean_s": {k: mean(k, lambda r: r["s"]) for k in VARIANTS},
        "reached": {k: int(sum(r[k]["reached"] for r in runs)) for k in VARIANTS},
        "runs": runs,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
