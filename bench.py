#!/usr/bin/env python3
"""Benchmark of the TV-regularised CT reconstruction hot path on one MI355X.

Workload (synthetic, seeded): 256^3 voxels, cone beam with 60 views over
360 degrees, flat detector 384 x 256 at pitch 1.5, source 1024 and detector
1536 from the centre, 24-ellipsoid phantom, 0.5 % Gaussian noise,
alpha = 3e-3, tau = 1e-4.  Method: UPN (Alg. 3) with FP32 vectors and FP64
reductions; the projector walks the rays on the fly; the backprojector is
the faster of the stored voxel-major A^T's product (built before the timed
region, its size and build time reported) and the on-the-fly gather through
the scan's symmetry, timed on the workload first (the choice is reported).

A "step" is one UPN iteration: gradient at y (backprojection + TV stencil),
projected trial step(s) with the projector's fused residual, the scalar
control and the extrapolation.  `value` is gradient evaluations per second
over exactly --steps iterations (inputs resident in HBM).  Beside it: the
same rate with the other backprojector; the time to a 1e-6 relative
gradient-map tolerance from x0 = 0 for UPN in FP32 and in FP64 (the metric's
two halves, their ratio, and the FP32 result's distance to the FP64 one),
and for GP in FP64 (the paper's plain method in plain precision; capped in
wall time); the live per-kernel durations (HIP events around each launch of
the timed solve) and the dominant kernel's roofline; the 32-problem batch,
the differentiated 64^3 form and the paper's own 64^3 experiment; and the
FP64 CPU oracle's gradient-evaluation rate on the host cores.

Before the timed region the tile shapes of the on-the-fly operators are
autotuned on the workload (the choice is reported), and a 1 GiB device copy
measures the attainable HBM rate for the roofline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-paper]
                       [--methods] [--gp64-iters N] [--gp64-seconds S]
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

# HBM bytes per launch, from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch) on the 256^3 cone workload, each scaled by what the counter reads
# for a 1 GiB device copy (FETCH_SIZE 524308 KiB: x 2; WRITE_SIZE 1048576 KiB:
# x 1).  An entry is reported only while the text of its source files is the
# one measured, and the projector's only at the measured ray tile
# (profiles/cone256_kernels_hbm_traffic_pmc.md).
MEASURED_TRAFFIC = [
    # project_kernel<float, cone, 2 columns, 8 or 4 waves> (z-fastest
    # companion): 2393131.5 + 105130.0 and 2428391.0 + 109564.7 KiB
    {"kernel": "project", "stored": None, "tile": (2, 8),
     "sources": ["paper_1105_4002_amd/csrc/project.hip",
                 "paper_1105_4002_amd/csrc/raywalk.hpp"],
     "sha256_prefix": "39eaafeffd2d100e", "bytes": (2 * 2393131.5 + 105130.0) * 1024},
    {"kernel": "project", "stored": None, "tile": (2, 4),
     "sources": ["paper_1105_4002_amd/csrc/project.hip",
                 "paper_1105_4002_amd/csrc/raywalk.hpp"],
     "sha256_prefix": "39eaafeffd2d100e", "bytes": (2 * 2428391.0 + 109564.7) * 1024},
    # backproject_sym_kernel<float, quarter turns, z mirror, 4 deep>: 49026.9 + 66366.9 KiB
    {"kernel": "backproject", "stored": False, "tile": None,
     "sources": ["paper_1105_4002_amd/csrc/backproject.hip",
                 "paper_1105_4002_amd/csrc/gather.hpp"],
     "sha256_prefix": "17b379376387c899", "bytes": (2 * 49026.9 + 66366.9) * 1024},
    # spmv_sym_kernel<float, quarter turns, z mirror>: 814996.4 + 77781.3 KiB
    {"kernel": "backproject", "stored": True, "tile": None,
     "sources": ["paper_1105_4002_amd/csrc/matrix.hip"], "sha256_prefix": "80160ee1be1d8553",
     "bytes": (2 * 814996.4 + 77781.3) * 1024},
]


def sources_sha(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, stored: bool, tile=None):
    """GB per launch measured for `kernel` in this form (backprojector from
    the stored A^T or on the fly; the projector's ray tile), or None when
    there is no such measurement or its sources have changed since."""
    for e in MEASURED_TRAFFIC:
        if e["kernel"] != kernel or (e["stored"] is not None and e["stored"] != stored):
            continue
        if e["tile"] is not None and tuple(tile or ()) != e["tile"]:
            continue
        if sources_sha(e["sources"]).startswith(e["sha256_prefix"]):
            return round(e["bytes"] / 1e9, 3)
    return None


FP64_VEC_PEAK = 78.6e12     # flop/s, MI355X FP64 vector (= FP32 without packed math)
# vector instruction issue: 256 CUs x 4 SIMDs x 16 lanes per clock at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 64 * 2.4e9   # lane-instructions/s
# vector instructions per voxel step of the projector's walk loop (count of the
# gfx950 code the build emits for the single-precision project_kernel of the
# column ray tiles on volumes under 2 GiB: 81 per iteration of four steps.
# Per step: 3 min for the segment end, the length, 2 compares, 5 selects and
# an add that pick the moving axis and its byte-offset step (the y and z
# moves from scalar lane-mask operations), 3 adds and 3 FMAs for the planes
# and next crossings, convert and accumulate; per iteration: the exit test
# (the step bound is scalar).  The row tiles' walk takes 44 per two.)
PROJECT_VALU_PER_STEP = 20.25


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_model(name: str, N: int, m: int, nnz: int, es: int, stored: bool):
    """Algorithmic work of one launch of each solver kernel (es = bytes per
    stored value).  Returns (bound, amount, unit, peak).

    The two ray kernels are gathers: per non-zero a_ij one value of the other
    vector is read (x for A, r for A^T), served by the caches or HBM.  The
    projector walks its rays on the fly and is held by instruction issue: its
    work is its vector instructions (PROJECT_VALU_PER_STEP per voxel step)
    against the issue rate.  The backprojector, streaming the stored A^T or
    gathering on the fly, is rated on the gather model of the product: es
    per non-zero (the value of r it reads) plus the volume written and the
    residual's compulsory read."""
    if name == "project":
        return "alu", PROJECT_VALU_PER_STEP * float(nnz), "T lane-instr/s", VALU_ISSUE_PEAK
    if name == "backproject":
        # both forms (stored A^T, on-the-fly gather) against the gather model
        return "hbm", es * float(nnz) + 2.0 * es * N, "GB/s", HBM_PEAK
    if name == "tv":
        return "hbm", es * 4.0 * N, "GB/s", HBM_PEAK       # y, x_ref, g in, g out
    if name == "trial":
        return "hbm", es * 3.0 * N, "GB/s", HBM_PEAK       # z, g in, xbar out
    if name == "extrapolate":
        return "hbm", es * 3.0 * (N + m), "GB/s", HBM_PEAK  # volume and residual, one launch
    if name == "transpose":
        return "hbm", es * 2.0 * N, "GB/s", HBM_PEAK       # volume in, y-fastest copy out
    raise KeyError(name)


def copy_bandwidth(torch, dev, reps: int = 10) -> float:
    """Device-to-device copy of 1 GiB timed with HIP events: the attainable
    HBM rate (GB/s, bytes read plus written) beside the spec-sheet peak."""
    src = torch.ones(2**28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * src.numel() * 4 * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    return gbs


def grad_eval_loop(tv, torch, G, b, x, w, n: int = 100, runs: int = 5) -> dict:
    """n back-to-back evaluations of phi and grad phi (tvreg_objective_grad)
    at x, timed with HIP events; the median over runs."""
    ws = tv.objective_workspace(G)
    g = G.empty_volume()
    tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
    rates = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
        e1.record()
        e1.synchronize()
        rates.append(n / (e0.elapsed_time(e1) / 1e3))
    rates.sort()
    return {"evals": n, "runs": runs, "grad_evals_per_s": round(rates[len(rates) // 2], 3),
            "ms_per_eval": round(1e3 / rates[len(rates) // 2], 4)}


def paper_leg(tv, synth, torch, dev, eps: float = 1e-8, max_iter: int = 20000) -> dict:
    """The paper's experiment (Sec. IV): 64^3, parallel beam with view
    directions over the unit sphere, 55 (many-view) and 19 (few-view) views of
    91^2 pixels, 1 % noise, alpha = 1e-2 (ellipsoids stand in for FORBILD).
    FP64 with the stored A^T and tuned shapes.  GP, GPBB and UPN run to the
    paper's stop test |G|/N <= eps (eq. 10, stop_mode 1); phi* is UPN at
    eps / 100, as in the paper.  Reported per method: iterations, seconds,
    status, and the relative gap (phi_k - phi*) / phi* after 10, 100, 500,
    1000, 2000 iterations and the first k where it falls below 1e-6."""
    out = {}
    for views in (55, 19):
        w = synth.cfg_paper(views)
        G = tv.Geometry(w.geom, tv.F64)
        xt = torch.from_numpy(w.phantom()).to(dev)
        ax = tv.project(G, xt)
        sigma = w.eta * torch.linalg.vector_norm(ax).item() / math.sqrt(ax.numel())
        b = (ax + sigma * torch.from_numpy(w.unit_noise()).to(dev)).float().double().contiguous()
        del ax
        G.attach_matrix()
        G.autotune(reps=5)
        common = dict(alpha=w.alpha, tau=w.tau, stop_mode=1)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        _, istar, _ = tv.solve(G, b, method=tv.UPN, eps=eps / 100, max_iter=10 * max_iter,
                               **common)
        torch.cuda.synchronize()
        phi_star = istar["phi"]
        case = {"views": views, "rays": w.geom.n_rays, "voxels": w.geom.n_voxels,
                "phi_star": phi_star, "phi_star_iters": istar["iters"],
                "phi_star_status": istar["stop_reason"],
                "phi_star_seconds": round(time.perf_counter() - s0, 3)}
        for meth, name in ((tv.UPN, "upn"), (tv.GPBB, "gpbb"), (tv.GP, "gp")):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            _, info, h = tv.solve(G, b, method=meth, eps=eps, max_iter=max_iter,
                                  hist_len=max_iter, **common)
            torch.cuda.synchronize()
            dt = time.perf_counter() - s0
            gap = [(p - phi_star) / phi_star for p in h["phi"]]
            first = next((k + 1 for k, v in enumerate(gap) if v <= 1e-6), None)
            case[name] = {"iters": info["iters"], "status": info["stop_reason"],
                          "seconds": round(dt, 3), "grad_evals": info["grad_evals"],
                          "func_evals": info["func_evals"],
                          "gap_at": {k: gap[k - 1] for k in (10, 100, 500, 1000, 2000)
                                     if k <= len(gap)},
                          "final_gap": gap[-1] if gap else None,
                          "first_iter_gap_below_1e-6": first}
        out[f"views{views}"] = case
        del G
    return out


def grad_eval_graph(tv, torch, G, b, x, w, n: int = 100, runs: int = 5) -> dict:
    """n evaluations of phi and grad phi captured in one HIP graph and
    replayed (each replay timed with HIP events; the median over runs)."""
    ws = tv.objective_workspace(G)
    g = G.empty_volume()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(n):
            tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
    rates = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        rates.append(n / (e0.elapsed_time(e1) / 1e3))
    rates.sort()
    del graph
    return {"evals": n, "runs": runs, "grad_evals_per_s": round(rates[len(rates) // 2], 3),
            "ms_per_eval": round(1e3 / rates[len(rates) // 2], 4)}


def gp64_leg(tv, torch, G, b, common: dict, tol: float, max_iter: int, stored: bool,
             chunk: int = 4000, max_seconds: float = 0.0) -> dict:
    """GP (eq. 6 with BT) in FP64 to the relative gradient-map tolerance, in
    chunks of `chunk` iterations so that progress is reported.  GP's only
    state is (x, L): a chunk starts from the previous chunk's x with L_bar =
    its last L and stops on |G| <= tol |G_0| written as the absolute test
    |G| / N <= tol |G_0| / N, so the chunks take exactly the steps of one
    uninterrupted run.  With max_seconds > 0 no chunk starts after that much
    wall time (the result then says not converged, with the |G| reached)."""
    if stored:
        G.attach_matrix()
    ws = tv.solve_workspace(G, tv.GP)
    x, L, iters, gm0, status, gm_rel = None, 1.0, 0, None, tv.ENOTCONV, None
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    while iters < max_iter:
        n = min(chunk, max_iter - iters)
        if gm0 is None:
            x, info, _ = tv.solve(G, b, method=tv.GP, eps=tol, max_iter=n, workspace=ws,
                                  **common)
            gm0 = info["gm_abs_over_N"] * G.N / info["gm_rel"] if info["gm_rel"] > 0 else 0.0
        else:
            x, info, _ = tv.solve(G, b, method=tv.GP, eps=tol * gm0 / G.N, stop_mode=1,
                                  max_iter=n, x0=x, L_bar=L, workspace=ws, **common)
        iters += info["iters"]  # a chunk's first iteration continues the previous one's
        L, status = info["L"], info["stop_reason"]
        gm_rel = info["gm_abs_over_N"] * G.N / gm0 if gm0 else 0.0
        log(f"  GP FP64: {iters} iterations, |G|/|G_0| = {gm_rel:.3e}, "
            f"{time.perf_counter() - s0:.1f} s")
        if status != tv.ENOTCONV:
            break
        if max_seconds > 0 and time.perf_counter() - s0 >= max_seconds:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - s0
    if stored:
        G.detach_matrix()
    return {"seconds": round(dt, 3), "iters": iters, "gm_rel": gm_rel, "status": status,
            "chunk": chunk}


def batch_leg(tv, synth, torch, dev, tol: float, max_iter: int, sequential: bool,
              stored: bool = False, tune: bool = True, probe_iters: int = 100):
    """The 32-problem batch (uneven sizes, views and alphas), FP32 UPN to tol:
    one tvreg_solve_batched call, and optionally the same problems one by one;
    with `stored`, every problem streams its stored A^T (built beforehand).
    With `tune`, the tile shapes are chosen first (outside the timing): each
    problem's own autotuned shapes or the defaults, whichever runs the first
    `probe_iters` rounds of the batch faster."""
    ws_ = synth.cfg_batch()
    geoms, bs = [], []
    for w in ws_:
        G64 = tv.Geometry(w.geom, tv.F64)
        ax = tv.project(G64, torch.from_numpy(w.phantom()).to(dev))
        sigma = w.eta * torch.linalg.vector_norm(ax).item() / math.sqrt(ax.numel())
        bs.append((ax + sigma * torch.from_numpy(w.unit_noise()).to(dev)).float().contiguous())
        del G64, ax
        geoms.append(tv.Geometry(w.geom, tv.F32))
    build_s = None
    if stored:
        torch.cuda.synchronize()
        m0 = time.perf_counter()
        for G in geoms:
            G.attach_matrix()
        torch.cuda.synchronize()
        build_s = round(time.perf_counter() - m0, 3)
    params = [dict(method=tv.UPN, alpha=w.alpha, tau=w.tau, eps=tol, max_iter=max_iter)
              for w in ws_]
    ws = tv.solve_batched_workspace(geoms, dev)
    tuned = None
    if tune:
        # Shapes are chosen for the batch as a whole: every problem's shapes
        # from its own autotune (timed alone), against the default shapes
        # for all, each timed over the first rounds of this batch.
        defaults = [G.tuning for G in geoms]
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        own = []
        for G in geoms:
            G.autotune(reps=3)
            own.append(G.tuning)
        probe = [dict(p, eps=0.0, max_iter=probe_iters) for p in params]

        def rounds_s(shapes):
            for G, sh in zip(geoms, shapes):
                G.set_tuning(*sh)
            tv.solve_batched(geoms, bs, probe, workspace=ws)
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            tv.solve_batched(geoms, bs, probe, workspace=ws)
            torch.cuda.synchronize()
            return time.perf_counter() - r0

        t_own, t_def = rounds_s(own), rounds_s(defaults)
        pick = own if t_own < t_def else defaults
        for G, sh in zip(geoms, pick):
            G.set_tuning(*sh)
        torch.cuda.synchronize()
        tuned = {"seconds": round(time.perf_counter() - a0, 3), "probe_rounds": probe_iters,
                 "per_problem_shapes_s": round(t_own, 4), "default_shapes_s": round(t_def, 4),
                 "chosen": "per_problem" if pick is own else "default",
                 "distinct_shapes": len(set(pick))}
    ws = tv.solve_batched_workspace(geoms, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos, status = tv.solve_batched(geoms, bs, params, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"problems": len(geoms), "voxels": int(sum(g.N for g in geoms)),
           "batched_seconds": round(dt, 3), "status": int(status),
           "iters_max": max(i["iters"] for i in infos),
           "grad_evals": int(sum(i["grad_evals"] for i in infos)),
           "converged": int(sum(1 for i in infos if i["stop_reason"] == tv.OK)),
           "shapes": tuned}
    if stored:
        out["stored_transpose_gib"] = round(sum(G.matrix_bytes for G in geoms) / 2**30, 3)
        out["stored_transpose_build_s"] = build_s
    if sequential:
        t0 = time.perf_counter()
        for G, b, p in zip(geoms, bs, params):
            tv.solve(G, b, **p)
        torch.cuda.synchronize()
        out["sequential_seconds"] = round(time.perf_counter() - t0, 3)
        out["speedup"] = round(out["sequential_seconds"] / dt, 3)
    return out


def unrolled_leg(tv, synth, torch, dev, reps: int = 3):
    """The differentiated form: 64^3, cone beam, 30 views, 96 x 96, K = 30
    unrolled UPN steps, forward + reverse pass in FP32 (checkpoints every 5),
    with the stored A^T and autotuned shapes."""
    w = synth.cfg_unrolled()
    G = tv.Geometry(w.geom, tv.F32)
    G.attach_matrix()
    G.autotune(reps=5)
    G64 = tv.Geometry(w.geom, tv.F64)
    xt = torch.from_numpy(w.phantom()).to(dev)
    ax = tv.project(G64, xt)
    sigma = w.eta * torch.linalg.vector_norm(ax).item() / math.sqrt(ax.numel())
    b = (ax + sigma * torch.from_numpy(w.unit_noise()).to(dev)).float().contiguous()
    xt32 = xt.float()
    tape = tv.unrolled_workspace(G, 30, 5, dev)
    xK, tape, L = tv.upn_unrolled_fwd(G, b, 30, w.alpha, tau=w.tau, tape=tape)
    tv.upn_unrolled_bwd(G, b, tape, 2.0 * (xK - xt32))
    torch.cuda.synchronize()
    tf = tb = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        xK, tape, _ = tv.upn_unrolled_fwd(G, b, 30, w.alpha, tau=w.tau, L_replay=L, tape=tape)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tv.upn_unrolled_bwd(G, b, tape, 2.0 * (xK - xt32))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tf += t1 - t0
        tb += t2 - t1
    return {"K": 30, "ckpt_every": 5, "forward_ms": round(1e3 * tf / reps, 2),
            "reverse_ms": round(1e3 * tb / reps, 2)}


def small_leg(tv, synth, torch, dev, tol: float) -> dict:
    """The small workloads on the GPU, stored A^T and default tile shapes:
    gradient evaluations per second (100 evaluations at x_true, FP32) and time
    to the relative gradient-map tolerance from x0 = 0 (UPN in FP32 and FP64;
    also GP and GPBB on parallel24, at most 5000 iterations).  Data: the
    projection of the phantom plus the seeded noise, as for the headline."""
    cases = [("parallel24", synth.cfg_small_parallel(), ["gp", "gpbb", "upn"]),
             ("cone64_a0.01", synth.cfg_cone64(1e-2), ["upn"]),
             ("cone64_a0.001", synth.cfg_cone64(1e-3), ["upn"]),
             ("cone64_30views", synth.cfg_unrolled(), ["upn"])]
    methods = {"gp": tv.GP, "gpbb": tv.GPBB, "upn": tv.UPN}
    out = {}
    for name, w, solves in cases:
        g = w.geom
        x_true = torch.from_numpy(w.phantom()).to(dev)
        G64, G32 = tv.Geometry(g, tv.F64), tv.Geometry(g, tv.F32)
        ax = tv.project(G64, x_true)
        sigma = w.eta * torch.linalg.vector_norm(ax).item() / math.sqrt(g.n_rays)
        b64 = ax + sigma * torch.from_numpy(w.unit_noise()).to(dev)
        b32 = b64.to(torch.float32).contiguous()
        G32.attach_matrix()
        G64.attach_matrix()
        x32 = x_true.to(torch.float32)
        for _ in range(5):
            tv.objective_grad(G32, b32, w.alpha, w.tau, x32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            tv.objective_grad(G32, b32, w.alpha, w.tau, x32)
        torch.cuda.synchronize()
        rec = {"grad_evals_per_s": round(100 / (time.perf_counter() - t0), 1)}
        for mth in solves:
            for label, G, bb in (("f32", G32, b32), ("f64", G64, b64)):
                ws = tv.solve_workspace(G, methods[mth])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info, _ = tv.solve(G, bb, method=methods[mth], alpha=w.alpha, tau=w.tau,
                                      eps=tol, max_iter=5000, workspace=ws)
                torch.cuda.synchronize()
                rec[f"time_to_tol_{mth}_{label}"] = {
                    "seconds": round(time.perf_counter() - t0, 3), "iters": info["iters"],
                    "status": info["stop_reason"]}
        log(f"  {name}: {rec}")
        out[name] = rec
        del G32, G64
    return out


def oracle_table(evals_only: bool) -> dict:
    """CPU oracle timings per workload (FP64, the host's OpenMP threads): gradient
    evaluations per second at x_true, and time to the 1e-6 relative gradient-map
    tolerance from x0 = 0 (GP, GPBB and UPN on parallel24; UPN on the 64^3 cone
    scans).  The 32-problem batch gets one gradient of every problem; its
    solves (about 38 000 gradient evaluations in all) are not run.  Touches no GPU."""
    import oracle
    import synth
    out = {"threads": oracle.num_threads(), "configs": {}}
    cases = [("parallel24", synth.cfg_small_parallel(), ["gp", "gpbb", "upn"]),
             ("cone64_a0.01", synth.cfg_cone64(1e-2), ["upn"]),
             ("cone64_a0.001", synth.cfg_cone64(1e-3), ["upn"]),
             ("cone64_30views", synth.cfg_unrolled(), ["upn"]),
             ("cone256", synth.cfg_cone256(), [])]
    methods = {"gp": oracle.GP, "gpbb": oracle.GPBB, "upn": oracle.UPN}
    for name, w, solves in cases:
        og = oracle.Geometry(w.geom)
        b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
        x = w.phantom()
        n, t0 = 0, time.perf_counter()
        while True:
            oracle.phi_grad(og, b, w.alpha, w.tau, x)
            n += 1
            if time.perf_counter() - t0 >= 3.0 or (n >= 1 and name == "cone256"):
                break
        rec = {"grad_evals_per_s": round(n / (time.perf_counter() - t0), 4)}
        log(f"oracle {name}: {rec['grad_evals_per_s']} gradient evals/s")
        if not evals_only:
            for mth in solves:
                t0 = time.perf_counter()
                _, info, _ = oracle.solve(og, b, method=methods[mth], alpha=w.alpha, tau=w.tau,
                                          eps=1e-6, max_iter=5000)
                rec[f"time_to_tol_{mth}"] = {"seconds": round(time.perf_counter() - t0, 2),
                                             "iters": info["iters"], "status": info["status"]}
                log(f"oracle {name} {mth}: {rec[f'time_to_tol_{mth}']}")
        out["configs"][name] = rec
    t0 = time.perf_counter()
    for w in synth.cfg_batch():
        og = oracle.Geometry(w.geom)
        b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
        oracle.phi_grad(og, b, w.alpha, w.tau, w.phantom())
    dt = time.perf_counter() - t0
    out["configs"]["batch32"] = {"one_gradient_of_each_s": round(dt, 2),
                                 "note": "includes building each problem's data"}
    log(f"oracle batch32: one gradient of each problem {dt:.1f} s")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--no-tol", action="store_true", help="skip the time-to-tolerance solve")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 UPN solve to tolerance (the metric's FP64 half)")
    ap.add_argument("--gp64-iters", type=int, default=100000,
                    help="GP in FP64 to --tol: at most this many iterations (0: skip)")
    ap.add_argument("--gp64-seconds", type=float, default=280.0,
                    help="GP in FP64: start no chunk of 4000 iterations after this many "
                         "seconds (0: no limit)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-matrix", action="store_true",
                    help="evaluate A^T on the fly in the headline solve (no stored A^T built)")
    ap.add_argument("--backprojector", choices=("auto", "stored", "on_the_fly"), default="auto",
                    help="the headline's backprojector: the faster of the two on the workload "
                         "(auto), or the one named")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the on-the-fly, batch and differentiated legs")
    ap.add_argument("--batch-seq", action="store_true",
                    help="also solve the batch problems one by one")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy of known size that "
                         "scales hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default tile shapes instead of autotuning them")
    ap.add_argument("--methods", action="store_true",
                    help="also time GP and GPBB (FP32 and FP64) to tolerance")
    ap.add_argument("--methods-max-iter", type=int, default=3000)
    ap.add_argument("--small", action="store_true",
                    help="also time the small workloads (parallel24, the 64^3 cone scans)")
    ap.add_argument("--oracle-table", action="store_true",
                    help="CPU only: time the FP64 oracle on every workload, on all host threads "
                         "and (in a child process) on one, and print that table instead")
    ap.add_argument("--oracle-evals-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper's 64^3 experiment (55 and 19 sphere views)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not an implemented mode.",
              file=sys.stderr)
        return 2

    if args.oracle_table or args.oracle_evals_only:
        table = oracle_table(args.oracle_evals_only)
        if args.oracle_table:
            import subprocess
            env = dict(os.environ, OMP_NUM_THREADS="1")
            log("the same gradient evaluations on one thread (child process)")
            child = subprocess.run([sys.executable, os.path.abspath(__file__),
                                    "--oracle-evals-only"], env=env, capture_output=True,
                                   text=True, check=True)
            one = json.loads(child.stdout.strip().splitlines()[-1])
            for name, rec in one["configs"].items():
                key = "grad_evals_per_s" if "grad_evals_per_s" in rec else "one_gradient_of_each_s"
                table["configs"][name][key + "_1thread"] = rec[key]
        print(json.dumps(table), flush=True)
        return 0

    import numpy as np
    import torch

    import paper_1105_4002_amd as tv
    import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(2**28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
    stored = not args.no_matrix and args.backprojector != "on_the_fly"
    matrix = None
    if stored:
        log("building the stored A^T")
        torch.cuda.synchronize()
        m0 = time.perf_counter()
        mnnz = G32.attach_matrix()
        torch.cuda.synchronize()
        matrix = {"gib": round(G32.matrix_bytes / 2**30, 3), "nnz": mnnz,
                  "build_s": round(time.perf_counter() - m0, 3),
                  "voxels_per_entry": G32.symmetry, "stored_bytes": G32.matrix_bytes}

    copy_gbs = copy_bandwidth(torch, dev)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    tuning = None
    if not args.no_tune:
        log("autotuning the on-the-fly operators' tile shapes")
        t = G32.autotune(reps=5)
        G64.set_tuning(*G32.tuning)
        tuning = {"project_tile_cols": t["project_tile_cols"],
                  "project_waves": t["project_waves"],
                  "backproject_depth": t["backproject_depth"],
                  "project_ms": round(t["project_ms"][(t["project_tile_cols"],
                                                       t["project_waves"])], 4),
                  # the best row tile (64 x 1 .. 8 x 8 rays per wave) and the
                  # best column tile (1 x 64, 2 x 32), each at its best height
                  "project_ms_row_tiles": round(min(v for (c, _), v in t["project_ms"].items()
                                                    if c >= 8), 4),
                  "project_ms_column_tiles": round(min(v for (c, _), v in
                                                       t["project_ms"].items() if c <= 2), 4),
                  "backproject_on_the_fly_ms": round(t["backproject_ms"][t["backproject_depth"]],
                                                     4)}
        log(f"  {tuning}")

    choice = None
    if stored:
        # the headline takes the faster backprojector: the stored A^T's
        # product or the on-the-fly gather (through the scan's symmetry)
        rr = torch.randn(w.geom.proj_shape, device=dev).float()
        times = {}
        for form in ("stored", "on_the_fly"):
            if form == "on_the_fly":
                G32.detach_matrix()
            xb = tv.backproject(G32, rr)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                tv.backproject(G32, rr, out=xb)
            e1.record()
            e1.synchronize()
            times[form] = e0.elapsed_time(e1) / 10
        del rr, xb
        stored = (times["stored"] < times["on_the_fly"] if args.backprojector == "auto"
                  else args.backprojector == "stored")
        if stored:
            G32.attach_matrix()
        choice = {"stored_ms": round(times["stored"], 4),
                  "on_the_fly_ms": round(times["on_the_fly"], 4),
                  "chosen": "stored" if stored else "on_the_fly", "rule": args.backprojector}
        log(f"backprojector: {choice}")

    log(f"warmup: {args.warmup} UPN iterations")
    xw, iw, _ = tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=max(args.warmup, 1),
                         workspace=ws32, **common)
    torch.cuda.synchronize()

    log(f"timed: {args.steps} UPN iterations")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xk, ik, _ = tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=args.steps, x0=xw,
                         L_bar=iw["L"], workspace=ws32, **common)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = ik["grad_evals"] / elapsed
    log(f"timed solve: {elapsed:.3f} s, {ik['grad_evals']} gradient evaluations, "
        f"{ik['func_evals']} trial evaluations")
    # per-kernel times: the same iterations again with the library's HIP-event
    # timing of each launch on (not part of the timed solve above: its events
    # and their readout between the line-search trials add host time per step)
    tv.profile_reset()
    tv.profile_enable(True)
    tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=args.steps, x0=xw, L_bar=iw["L"],
             workspace=ws32, **common)
    torch.cuda.synchronize()
    tv.profile_enable(False)
    stats = tv.profile_stats()

    kernels = {}
    for name, (cnt, ms) in stats.items():
        if cnt:
            bound, amount, unit, peak = kernel_model(name, N, m, nnz, 4, stored)
            avg = ms / cnt / 1e3
            kernels[name] = {"launches": cnt, "avg_ms": round(ms / cnt, 4),
                             "total_ms": round(ms, 3), "bound": bound,
                             "frac": round(amount / avg / peak, 4)}
            if name == "project":
                # beside the issue rate: 7 flops per voxel step (3-way min,
                # length, two FMAs) against the FP64 vector peak, and the
                # gather model (4 B per non-zero + the residual's 8 B per ray)
                kernels[name]["flop_frac"] = round(7.0 * nnz / avg / FP64_VEC_PEAK, 4)
                kernels[name]["gather_model_hbm_frac"] = round(
                    (4.0 * nnz + 8.0 * m) / avg / HBM_PEAK, 4)
            if name == "backproject" and stored and matrix:
                # the stored layout's own stream: value + key per stored
                # entry (padding included), r, the volume
                lay = matrix["stored_bytes"] + 4.0 * (m + N)
                kernels[name]["stored_layout_GBps"] = round(lay / avg / 1e9, 1)
                kernels[name]["compulsory_hbm_frac"] = round(4.0 * (m + 2 * N) / avg / HBM_PEAK, 4)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    bound, amount, unit, peak = kernel_model(dom, N, m, nnz, 4, stored)
    avg_s = kernels[dom]["avg_ms"] / 1e3
    scale = 1e9 if unit == "GB/s" else 1e12
    tile = G32.tuning[:2]
    roofline = {"kernel": dom, "bound": bound, "achieved": round(amount / avg_s / scale, 3),
                "peak": peak / scale, "unit": unit, "frac": round(amount / avg_s / peak, 4),
                "traffic": measured_traffic(dom, stored, tile)}
    if bound == "hbm":
        roofline["copy_peak"] = round(copy_gbs, 1)
        roofline["frac_of_copy"] = round(amount / avg_s / 1e9 / copy_gbs, 4)
    if roofline["traffic"] is not None:
        roofline["traffic_unit"] = "GB per launch"
        # the bytes the kernel must move: its own model for an HBM-bound
        # kernel; for the projector the gather model (4 B per non-zero, the
        # residual's 8 B per ray)
        roofline["algorithmic_GB"] = round(
            (amount if bound == "hbm" else 4.0 * nnz + 8.0 * m) / 1e9, 3)
    for name in ("project", "backproject"):
        if name in kernels:
            t_gb = measured_traffic(name, stored, tile)
            if t_gb is not None:
                kernels[name]["traffic_GB"] = t_gb
                kernels[name]["traffic_GBps"] = round(t_gb / (kernels[name]["avg_ms"] / 1e3), 1)

    result = {
        "metric": "gradient evals/sec + time to 1e-6 gradient-map tol, 256^3 UPN FP32 vs FP64",
        "value": round(value, 3), "unit": "gradient evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cone256: 256^3 voxels, cone beam 60 views/360 deg, detector "
                               "384x256 @1.5, R=1024, SDD=1536, 24 ellipsoids, 0.5% noise, "
                               "alpha=3e-3, tau=1e-4; UPN, FP32 vectors + FP64 reductions",
                   "operators": ("projector on the fly, backprojector from the stored A^T"
                                 if stored else
                                 "both on the fly (the backprojector through the scan's "
                                 "symmetry)"),
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
    }
    if matrix:
        result["stored_transpose"] = matrix
    if choice:
        result["backprojector"] = choice
    if tuning:
        result["tuning"] = tuning
    result["hbm_copy_GBps"] = round(copy_gbs, 1)

    if not args.no_legs:
        log("100 gradient evaluations at x_true (median of 5)")
        result["grad_eval_loop"] = grad_eval_loop(tv, torch, G32, b32, x_true.float(), w)
        log(f"  {result['grad_eval_loop']}")
        log("100 gradient evaluations captured in one HIP graph (median of 5 replays)")
        result["grad_eval_graph"] = grad_eval_graph(tv, torch, G32, b32, x_true.float(), w)
        log(f"  {result['grad_eval_graph']}")

    if matrix and not args.no_legs:
        # the same solve with the other backprojector
        other = "on_the_fly" if stored else "with_stored_transpose"
        log(f"same solve {other.replace('_', ' ')}: {args.steps} UPN iterations")
        if stored:
            G32.detach_matrix()
        else:
            G32.attach_matrix()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, i0, _ = tv.solve(G32, b32, method=tv.UPN, eps=0.0, max_iter=args.steps, x0=xw,
                            L_bar=iw["L"], workspace=ws32, **common)
        torch.cuda.synchronize()
        d0 = time.perf_counter() - t0
        result[other] = {"value": round(i0["grad_evals"] / d0, 3),
                         "ms_per_step": round(1e3 * d0 / args.steps, 4)}
        if stored:
            G32.attach_matrix()
        else:
            G32.detach_matrix()

    x_tol = {}
    if not args.no_tol:
        for label, G, bb in [("f32", G32, b32)] + ([] if args.no_fp64 else [("f64", G64, b64)]):
            log(f"time to tolerance {args.tol:g}: UPN {label}")
            if label == "f64" and stored:
                G.attach_matrix()
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
            x_tol[label] = xs.double()
            if label == "f64":
                del ws
                if stored:
                    G.detach_matrix()
        if "f64" in x_tol:
            # the FP32 result against the FP64 one at the same tolerance: the
            # precision's share of the error (both carry the tolerance's)
            d = x_tol["f32"] - x_tol["f64"]
            result["time_to_tol_upn_f32"]["vs_f64"] = {
                "rel_l2": float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(x_tol["f64"])),
                "max_abs": float(d.abs().max())}
            result["ratios"] = {"upn_f64_over_upn_f32_seconds": round(
                result["time_to_tol_upn_f64"]["seconds"] / result["time_to_tol_upn_f32"]["seconds"], 3)}
        x_tol.clear()
    if not args.no_legs:
        log("32-problem batch, FP32 UPN to 1e-6")
        result["batch32"] = batch_leg(tv, synth, torch, dev, 1e-6, 5000, args.batch_seq,
                                      tune=not args.no_tune)
        log(f"  {result['batch32']}")
        log("32-problem batch with stored A^T, FP32 UPN to 1e-6")
        result["batch32_stored"] = batch_leg(tv, synth, torch, dev, 1e-6, 5000, args.batch_seq,
                                             stored=True, tune=not args.no_tune)
        log(f"  {result['batch32_stored']}")
        log("differentiated form: 64^3, K = 30")
        result["unrolled64"] = unrolled_leg(tv, synth, torch, dev)
        log(f"  {result['unrolled64']}")
    if args.methods:
        for meth, name in ((tv.GPBB, "gpbb"), (tv.GP, "gp")):
            for label, G, bb in (("f32", G32, b32), ("f64", G64, b64)):
                log(f"time to tolerance {args.tol:g}: {name} {label}")
                if label == "f64" and stored:
                    G.attach_matrix()
                ws = tv.solve_workspace(G, meth)
                torch.cuda.synchronize()
                s0 = time.perf_counter()
                xs, info, _ = tv.solve(G, bb, method=meth, eps=args.tol,
                                       max_iter=args.methods_max_iter, workspace=ws, **common)
                torch.cuda.synchronize()
                dt = time.perf_counter() - s0
                result[f"time_to_tol_{name}_{label}"] = {
                    "seconds": round(dt, 3), "iters": info["iters"],
                    "grad_evals": info["grad_evals"], "func_evals": info["func_evals"],
                    "gm_rel": info["gm_rel"], "status": info["stop_reason"]}
                log(f"  {dt:.2f} s, {info['iters']} iterations, status {info['stop_reason']}")
                del ws
                if label == "f64" and stored:
                    G.detach_matrix()
    if args.small:
        log(f"small workloads: gradient evals/s and time to {args.tol:g}")
        result["small"] = small_leg(tv, synth, torch, dev, args.tol)
    if not args.no_paper:
        log("the paper's experiment: 64^3, 55 and 19 views over the sphere, GP/GPBB/UPN FP64")
        result["paper_experiment"] = paper_leg(tv, synth, torch, dev)
        log(f"  {result['paper_experiment']}")
    if args.gp64_iters > 0:
        log(f"GP FP64 (the paper's plain method, plain precision) to {args.tol:g}, "
            f"at most {args.gp64_iters} iterations")
        result["gp_f64"] = gp64_leg(tv, torch, G64, b64, common, args.tol, args.gp64_iters,
                                    stored, max_seconds=args.gp64_seconds)
        if "time_to_tol_upn_f32" in result and result["gp_f64"]["status"] == tv.OK:
            result.setdefault("ratios", {})["gp_f64_over_upn_f32_seconds"] = round(
                result["gp_f64"]["seconds"] / result["time_to_tol_upn_f32"]["seconds"], 2)

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
