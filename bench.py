#!/usr/bin/env python3
"""Benchmark of the TV-regularised CT reconstruction hot path on one MI355X.

Workload (synthetic, seeded): 256^3 voxels, cone beam with 60 views over
360 degrees, flat detector 384 x 256 at pitch 1.5, source 1024 and detector
1536 from the centre, 24-ellipsoid phantom, 0.5 % Gaussian noise,
alpha = 3e-3, tau = 1e-4.  Method: UPN (Alg. 3) with FP32 vectors and FP64
reductions.

A "step" is one UPN iteration: gradient at y (gather backprojection + TV
stencil), projected trial step(s) with the projector's fused residual, the
scalar control and the extrapolation.  `value` is gradient evaluations per
second over exactly --steps iterations (inputs resident in HBM).  Beside it:
the time to a 1e-6 relative gradient-map tolerance from x0 = 0, the live
per-kernel durations (HIP events around each launch of the timed solve), the
dominant kernel's roofline, and the FP64 CPU oracle's gradient-evaluation
rate on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--fp64] [--gp64-iters N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12           # bytes/s, MI355X HBM3E
FP64_VEC_PEAK = 78.6e12     # flop/s, MI355X FP64 vector (= FP32 without packed math)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_model(name: str, N: int, m: int, nnz: int, es: int):
    """Algorithmic work of one launch of each solver kernel (FP32 storage,
    es = 4 bytes).  Returns (bound, amount, unit, peak)."""
    if name == "project":
        # 7 flops per (ray, voxel) step of the walk: 3-way min, length,
        # accumulate (FMA = 2), next-crossing update (FMA = 2)
        return "alu", 7.0 * nnz, "TFLOP/s", FP64_VEC_PEAK
    if name == "backproject":
        # 10 flops per (voxel, ray) pair: two z-plane parameters (2 FMA),
        # max, min, length, |D| scale, accumulate (FMA)
        return "alu", 10.0 * nnz, "TFLOP/s", FP64_VEC_PEAK
    if name == "tv":
        return "hbm", es * 4.0 * N, "GB/s", HBM_PEAK       # y, x_ref, g in, g out
    if name == "trial":
        return "hbm", es * 3.0 * N, "GB/s", HBM_PEAK       # z, g in, xbar out
    if name == "extrapolate":
        return "hbm", es * 3.0 * (N + m) / 2.0, "GB/s", HBM_PEAK  # mean of the N and m launches
    if name == "transpose":
        return "hbm", es * 2.0 * N, "GB/s", HBM_PEAK       # volume in, y-fastest copy out
    raise KeyError(name)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--no-tol", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--fp64", action="store_true", help="also time UPN in FP64 to tolerance")
    ap.add_argument("--gp64-iters", type=int, default=0,
                    help="also run GP in FP64 for up to this many iterations")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not an implemented mode.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1105_4002_amd as tv
    import synth

    dev = torch.device("cuda:0")
    w = synth.cfg_cone256()
    g = w.geom
    N, m = g.n_voxels, g.n_rays
    with open(os.path.join(ROOT, "tests", "golden", "operator_nnz.json")) as fh:
        nnz = json.load(fh)["cone256"]["nnz"]

    log("generating phantom and noise")
    x_true = torch.from_numpy(w.phantom()).to(dev)
    z = torch.from_numpy(w.unit_noise()).to(dev)
    G64 = tv.Geometry(g, tv.F64)
    G32 = tv.Geometry(g, tv.F32)
    ax = tv.project(G64, x_true)
    sigma = w.eta * torch.linalg.vector_norm(ax).item() / math.sqrt(m)
    b32 = (ax + sigma * z).to(torch.float32).contiguous()
    b64 = b32.to(torch.float64)
    del ax, z
    torch.cuda.synchronize()
    ws32 = tv.solve_workspace(G32, tv.UPN)
    common = dict(alpha=w.alpha, tau=w.tau)

    log(f"warmup: {args.warmup} UPN iterations")
    xw, iw, _ = tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=max(args.warmup, 1),
                         workspace=ws32, **common)
    torch.cuda.synchronize()

    log(f"timed: {args.steps} UPN iterations")
    tv.profile_reset()
    tv.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xk, ik, _ = tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=args.steps, x0=xw,
                         L_bar=iw["L"], workspace=ws32, **common)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tv.profile_enable(False)
    stats = tv.profile_stats()
    elapsed = t1 - t0
    value = ik["grad_evals"] / elapsed
    log(f"timed solve: {elapsed:.3f} s, {ik['grad_evals']} gradient evaluations, "
        f"{ik['func_evals']} trial evaluations")

    kernels = {}
    for name, (cnt, ms) in stats.items():
        if cnt:
            bound, amount, unit, peak = kernel_model(name, N, m, nnz, 4)
            avg = ms / cnt / 1e3
            kernels[name] = {"launches": cnt, "avg_ms": round(ms / cnt, 4),
                             "total_ms": round(ms, 3), "bound": bound,
                             "frac": round(amount / avg / peak, 4)}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    bound, amount, unit, peak = kernel_model(dom, N, m, nnz, 4)
    avg_s = kernels[dom]["avg_ms"] / 1e3
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    roofline = {"kernel": dom, "bound": bound, "achieved": round(amount / avg_s / scale, 3),
                "peak": peak / scale, "unit": unit, "frac": round(amount / avg_s / peak, 4),
                "traffic": None}

    result = {
        "metric": "gradient evals/sec + time to 1e-6 gradient-map tol, 256^3 UPN FP32 vs FP64",
        "value": round(value, 3), "unit": "gradient evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cone256: 256^3 voxels, cone beam 60 views/360 deg, detector "
                               "384x256 @1.5, R=1024, SDD=1536, 24 ellipsoids, 0.5% noise, "
                               "alpha=3e-3, tau=1e-4; UPN, FP32 vectors + FP64 reductions",
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
    }

    if not args.no_tol:
        for label, G, bb in [("f32", G32, b32)] + ([("f64", G64, b64)] if args.fp64 else []):
            log(f"time to tolerance {args.tol:g}: UPN {label}")
            ws = ws32 if label == "f32" else tv.solve_workspace(G, tv.UPN)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            xs, info, _ = tv.solve(G, bb, method=tv.UPN, eps=args.tol, max_iter=args.max_iter,
                                   workspace=ws, **common)
            torch.cuda.synchronize()
            dt = time.perf_counter() - s0
            result[f"time_to_tol_upn_{label}"] = {
                "seconds": round(dt, 3), "iters": info["iters"],
                "grad_evals": info["grad_evals"], "func_evals": info["func_evals"],
                "gm_rel": info["gm_rel"], "status": info["stop_reason"],
                "grad_evals_per_s": round(info["grad_evals"] / dt, 3)}
            log(f"  {dt:.2f} s, {info['iters']} iterations, status {info['stop_reason']}")
            if label == "f64":
                del ws
    if args.gp64_iters > 0:
        log(f"GP FP64 for up to {args.gp64_iters} iterations")
        ws = tv.solve_workspace(G64, tv.GP)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        xs, info, _ = tv.solve(G64, b64, method=tv.GP, eps=args.tol, max_iter=args.gp64_iters,
                               workspace=ws, **common)
        torch.cuda.synchronize()
        dt = time.perf_counter() - s0
        result["gp_f64"] = {"seconds": round(dt, 3), "iters": info["iters"],
                            "gm_rel": info["gm_rel"], "status": info["stop_reason"]}

    if not args.no_cpu:
        import oracle
        log("CPU oracle baseline (FP64 gradient evaluations of the same workload)")
        xh = x_true.cpu().numpy()
        bh = b64.cpu().numpy()
        n = 0
        c0 = time.perf_counter()
        while True:
            oracle.phi_grad(g, bh, w.alpha, w.tau, xh)
            n += 1
            if time.perf_counter() - c0 >= args.cpu_seconds or n >= 20:
                break
        cdt = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(n / cdt, 5), "unit": "gradient evals/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": f"{n} full FP64 gradient evaluations of the 256^3 "
                                            f"workload ({cdt:.1f} s)"}

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
