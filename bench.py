#!/usr/bin/env python3
"""Benchmark: time to 1e-10 relative residual for block COCR with residual
orthonormalization (Algorithm 3), mixed precision vs FP64, on the 3D
Helmholtz operator (7-point, 128^3 interior grid, n = 2,097,152,
nnz = 14,581,760, k h = 0.25, 2% damping) with p = 32 complex Gaussian
right-hand sides; plus the standalone operator application (SpMM) as a
fraction of HBM peak.

One step = one FP64 solve to 1e-10 and one mixed-precision solve to 1e-10 of
the same system, inputs resident in HBM.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--N 128] [--p 32]
                       [--no-cpu-baseline] [--spmm-reps R]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmm_bytes(n: int, nnz: int, p: int, cbytes: int, colind: bool = True) -> int:
    """Algorithmic bytes of Y = A Z: A once (values + int32 row pointers, and
    the int32 column indices unless the pattern is a verified grid stencil,
    whose product does not read them), Z read once, Y written once."""
    return nnz * (cbytes + (4 if colind else 0)) + 4 * (n + 1) + 2 * n * p * cbytes


# What the standalone product's counters depend on: the 2.5D kernel's sources
# and its launch code (the grid-stencil branch of apply_op in solver.hip).
SPMM_SOURCES = ["paper_1601_05362_amd/csrc/grid.hpp", "paper_1601_05362_amd/csrc/common.hpp",
                ("paper_1601_05362_amd/csrc/solver.hip", "        // grid-stencil pattern: 2.5D blocked product",
                 "    if (A.kind == BLK_OP_CSR) {")]
TRAFFIC_PROFILE = "profiles/k_spmm_c128_p32_helmholtz3d_128.md"


def source_hash(paths) -> str:
    """Hash of the code (comments and whitespace removed) of the given files or
    (file, begin marker, end marker) regions."""
    import hashlib
    import re

    h = hashlib.sha256()
    for item in paths:
        rel, begin, end = item if isinstance(item, tuple) else (item, None, None)
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            data = f.read()
        if begin is not None:
            i = data.index(begin)
            data = data[i:data.index(end, i)]
        data = re.sub(r"/\*.*?\*/", " ", data, flags=re.S)
        data = re.sub(r"//[^\n]*", " ", data)
        h.update(" ".join(data.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the SpMM from the committed counter summary,
    or None if the summary is missing or was taken on different kernel
    sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    want = source_hash(SPMM_SOURCES)
    fields = dict(line.split(":", 1) for line in txt.splitlines() if line.startswith("traffic_"))
    if fields.get("traffic_source_hash", "").strip() != want:
        return None
    try:
        return int(fields["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def time_spmm(pkg, torch, A, Z, reps: int, c64: bool) -> float:
    """Average duration (s) of one standalone SpMM launch, from HIP events
    recorded on the stream the kernels are launched on."""
    stream = torch.cuda.current_stream()
    Y = torch.empty_like(Z)
    fn = (lambda: pkg.blk_spmm_c(A, Z, out=Y)) if c64 else (lambda: pkg.blk_spmm_z(A, Z, out=Y))
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def per_iteration(pkg, torch, fn, A, B, short: int, long: int) -> float:
    """Seconds per iteration of an FP64 solve: (time of `long` iterations -
    time of `short`) / (long - short), so set-up and the final residual drop
    out.  The tolerance is unreachable, so every run does its full count."""
    t = {}
    for it in (short, long):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(A, B, tol=1e-300, maxit=it)
        torch.cuda.synchronize()
        t[it] = time.perf_counter() - t0
    return (t[long] - t[short]) / (long - short)


def cpu_baseline(Acsr, B, fp64_iters: int, sample_iters: int):
    """The oracle (numpy/scipy FP64) on a bounded sample: start-up plus
    `sample_iters` iterations of block COCR with residual orthonormalization,
    scaled to the GPU's FP64 iteration count."""
    from oracle import blk_oracle as O

    try:
        from threadpoolctl import threadpool_info

        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    O.bl_cocr_rq(Acsr, B, tol=1e-30, maxit=0)
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.bl_cocr_rq(Acsr, B, tol=1e-30, maxit=sample_iters)
    t_run = time.perf_counter() - t0
    per_iter = max(t_run - t_init, 1e-9) / sample_iters
    est = t_init + per_iter * fp64_iters
    return {
        "value": round(est, 3),
        "unit": "s",
        "cores": int(cores),
        "kind": "oracle",
        "sample": (f"start-up + {sample_iters} iterations of the numpy/scipy FP64 oracle "
                   f"bl_cocr_rq on the same n={Acsr.n}, p={B.shape[1]} system "
                   f"({per_iter:.2f} s/iteration, start-up {t_init:.2f} s), scaled to the "
                   f"GPU FP64 iteration count {fp64_iters}"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="interior grid points per axis")
    ap.add_argument("--p", type=int, default=32, help="right-hand sides")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--refine", type=int, default=2,
                    help="restarts allowed when the true residual lags the monitored one")
    ap.add_argument("--spmm-reps", type=int, default=50)
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--no-per-iter", action="store_true",
                    help="skip the per-iteration timings of the p = 32, p = 8 and 2D cases")
    ap.add_argument("--dense", type=int, default=0, metavar="N",
                    help="also time the dense Green's-function product at n = N (p as above)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the solver is a "
                          "single-GPU library (multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1601_05362_amd as pkg
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, p = args.N, args.p
    t0 = time.perf_counter()
    A = W.config2_operator(N)
    B = W.config2_rhs(A.n, p)
    log(f"[bench] inputs n={A.n} nnz={A.nnz} p={p} built in {time.perf_counter() - t0:.1f}s")
    Ad = pkg.CsrOperator.from_arrays(A.rowptr, A.colind, A.val, device=dev).analyze()
    grid_path = Ad.structure == pkg._capi.BLK_STRUCT_GRID
    log(f"[bench] operator pattern: {'grid stencil ' + str(Ad.grid) if grid_path else 'general CSR'}")
    Bd = torch.as_tensor(B, device=dev)
    X = torch.empty_like(Bd)
    torch.cuda.synchronize()

    # --- standalone SpMM (the dominant kernel) --------------------------------
    Zd = torch.as_tensor(W.cgauss(A.n, p, seed=5), device=dev)
    t_spmm = time_spmm(pkg, torch, Ad, Zd, args.spmm_reps, c64=False)
    b64 = spmm_bytes(A.n, A.nnz, p, 16, colind=not grid_path)
    Zc = Zd.to(torch.complex64)
    t_spmm32 = time_spmm(pkg, torch, Ad, Zc, args.spmm_reps, c64=True)
    b32 = spmm_bytes(A.n, A.nnz, p, 8, colind=not grid_path)
    gbs64, gbs32 = b64 / t_spmm / 1e9, b32 / t_spmm32 / 1e9
    log(f"[bench] spmm c128 p={p}: {t_spmm * 1e3:.3f} ms, {gbs64:.0f} GB/s ({gbs64 / HBM_PEAK_GBS:.1%} of peak); "
        f"c64: {t_spmm32 * 1e3:.3f} ms, {gbs32:.0f} GB/s ({gbs32 / HBM_PEAK_GBS:.1%})")
    # the same operator with p = 8 columns
    Z8 = torch.as_tensor(W.cgauss(A.n, 8, seed=6), device=dev)
    t_spmm8 = time_spmm(pkg, torch, Ad, Z8, args.spmm_reps, c64=False)
    b8 = spmm_bytes(A.n, A.nnz, 8, 16, colind=not grid_path)
    gbs8 = b8 / t_spmm8 / 1e9
    log(f"[bench] spmm c128 p=8: {t_spmm8 * 1e3:.3f} ms, {gbs8:.0f} GB/s ({gbs8 / HBM_PEAK_GBS:.1%})")
    del Z8
    # a plain copy of known size: the calibration point for HBM byte counters
    Yc = torch.empty_like(Zd)
    for _ in range(3):
        Yc.copy_(Zd)
    torch.cuda.synchronize()
    del Zd, Zc, Yc

    # --- optional: the dense Green's-function operator (second experiment) -----
    dense = None
    if args.dense:
        nd = args.dense
        t0 = time.perf_counter()
        Ah = W.greens_sphere(nd, 2.0 * math.pi * 8.0)
        Dd = pkg.DenseOperator(torch.as_tensor(Ah, device=dev))
        del Ah
        Zd = torch.as_tensor(W.cgauss(nd, p, seed=5), device=dev)
        Yd = torch.empty_like(Zd)
        log(f"[bench] dense operator n={nd} built in {time.perf_counter() - t0:.1f}s")
        stream = torch.cuda.current_stream()
        pkg.blk_spmm_z(Dd, Zd, out=Yd)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            pkg.blk_spmm_z(Dd, Zd, out=Yd)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        tf = 8.0 * nd * nd * p / (ms * 1e-3) / 1e12
        dense = {"n": nd, "p": p, "ms": round(ms, 4), "TFLOPs": round(tf, 2),
                 "frac_fp64_peak": round(tf / 78.6, 4),
                 "A_GBs": round(16.0 * nd * nd / (ms * 1e-3) / 1e9, 1)}
        log(f"[bench] dense c128 product n={nd} p={p}: {ms:.3f} ms, {tf:.1f} TFLOP/s")
        # the complex64 product of the mixed form's inner solves (FP32 matrix cores)
        Z32, Y32 = Zd.to(torch.complex64), Yd.to(torch.complex64)
        pkg.blk_spmm_c(Dd, Z32, out=Y32)
        e0.record(stream)
        for _ in range(5):
            pkg.blk_spmm_c(Dd, Z32, out=Y32)
        e1.record(stream)
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1) / 5
        tf32 = 8.0 * nd * nd * p / (ms32 * 1e-3) / 1e12
        dense["c64"] = {"ms": round(ms32, 4), "TFLOPs": round(tf32, 2),
                        "frac_fp32_peak": round(tf32 / 157.3, 4),
                        "A_GBs": round(8.0 * nd * nd / (ms32 * 1e-3) / 1e9, 1)}
        log(f"[bench] dense c64 product n={nd} p={p}: {ms32:.3f} ms, {tf32:.1f} TFLOP/s")
        del Dd, Z32, Y32, Zd, Yd
        torch.cuda.synchronize()

    # --- solves -----------------------------------------------------------------
    def step():
        out = {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = pkg.blk_cocr_solve(Ad, Bd, tol=args.tol, maxit=args.maxit, refine=args.refine, out=X)
        torch.cuda.synchronize()
        out["fp64"] = (time.perf_counter() - t, r)
        log(f"[bench]   fp64: {out['fp64'][0]:.3f}s iters={r.iters} status={r.status_name} trr={r.true_relres:.2e}")
        if not args.skip_mixed:
            t = time.perf_counter()
            r2 = pkg.blk_cocr_solve(Ad, Bd, tol=args.tol, maxit=args.maxit, precision="mixed",
                                    refine=args.refine, out=X)
            torch.cuda.synchronize()
            out["mixed"] = (time.perf_counter() - t, r2)
            log(f"[bench]   mixed: {out['mixed'][0]:.3f}s iters={r2.iters} status={r2.status_name} trr={r2.true_relres:.2e}")
        return out

    for w in range(args.warmup):
        log(f"[bench] warmup step {w}")
        step()
    torch.cuda.synchronize()
    results = []
    t_all = time.perf_counter()
    for k in range(args.steps):
        log(f"[bench] timed step {k}")
        results.append(step())
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all

    fp64_s = float(np.median([r["fp64"][0] for r in results]))
    rf = results[-1]["fp64"][1]
    mixed_s = float(np.median([r["mixed"][0] for r in results])) if not args.skip_mixed else None
    rm = results[-1]["mixed"][1] if not args.skip_mixed else None

    # --- time per FP64 iteration of every case (outside the timed region) -------
    per_iter = {}
    if not args.no_per_iter:
        solvers = (("cocr_rq", pkg.blk_cocr_solve), ("cocg_rq", pkg.blk_cocg_solve))
        for pq in sorted({p, 8}, reverse=True):
            Bq = torch.as_tensor(W.config2_rhs(A.n, pq), device=dev)
            for name, fn in solvers:
                per_iter[f"{N}^3_p{pq}_{name}_ms"] = round(
                    per_iteration(pkg, torch, fn, Ad, Bq, 10, 110) * 1e3, 4)
            del Bq
        A1, B1 = W.config1()
        A1d = pkg.CsrOperator.from_arrays(A1.rowptr, A1.colind, A1.val, device=dev)
        B1d = torch.as_tensor(B1, device=dev)
        for name, fn in solvers:
            per_iter[f"64^2_p4_{name}_us"] = round(per_iteration(pkg, torch, fn, A1d, B1d, 20, 420) * 1e6, 2)
        log(f"[bench] per iteration: {per_iter}")

    line = {
        "metric": "time to 1e-10 rel. residual, mixed vs FP64, n=2.1M p=32; SpMM % HBM peak",
        "value": round(mixed_s if mixed_s is not None else fp64_s, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64+f64" if mixed_s is not None else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"3D Helmholtz 7-point FD, {N}^3 interior grid (n={A.n}, nnz={A.nnz}), "
                         f"k h=0.25, 2% damping, complex128 CSR; p={p} complex Gaussian RHS (seed 1); "
                         f"bl_cocr_rq to {args.tol:g} relative residual, FP64 and mixed "
                         f"(complex64 inner solves, FP64 refinement)"),
            "n": A.n, "nnz": A.nnz, "p": p, "tol": args.tol, "refine": args.refine,
        },
        "fp64_s": round(fp64_s, 4),
        "fp64_iters": rf.iters,
        "fp64_status": rf.status_name,
        "fp64_true_relres": rf.true_relres,
        "fp64_ms_per_iter": round(fp64_s / max(rf.iters, 1) * 1e3, 4),
        "mixed_s": round(mixed_s, 4) if mixed_s is not None else None,
        "mixed_iters": rm.iters if rm is not None else None,
        "mixed_status": rm.status_name if rm is not None else None,
        "mixed_true_relres": rm.true_relres if rm is not None else None,
        "mixed_over_fp64": round(mixed_s / fp64_s, 3) if mixed_s is not None else None,
        "spmm_c128_ms": round(t_spmm * 1e3, 4),
        "spmm_c128_GBs": round(gbs64, 1),
        "spmm_c64_ms": round(t_spmm32 * 1e3, 4),
        "spmm_c64_GBs": round(gbs32, 1),
        "spmm_c128_p8_ms": round(t_spmm8 * 1e3, 4),
        "spmm_c128_p8_GBs": round(gbs8, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": (f"k_spmm_grid complex128 p={p} (2.5D, grid-stencil pattern)" if grid_path
                       else f"k_spmm complex128 p={p}"),
            "achieved": round(gbs64, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs64 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(),
            "algorithmic_bytes_per_launch": b64,
            "avg_launch_ms": round(t_spmm * 1e3, 4),
        },
        "cpu_baseline": None,
        "dense_product": dense,
        "fp64_per_iteration": per_iter or None,
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        del Ad, Bd, X
        torch.cuda.empty_cache()
        line["cpu_baseline"] = cpu_baseline(A, B, rf.iters, args.cpu_sample_iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
