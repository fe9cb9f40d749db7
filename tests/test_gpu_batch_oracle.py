"""The batched solve (tvreg_solve_batched) against the FP64 oracle directly,
not through tvreg_solve: the device control step (BT test of Alg. 2, the mu
estimate of eq. 9, theta and beta of Alg. 3, the stop test of eq. 10) and the
grouped kernels must take the oracle's decisions.

* FP64, five uneven problems in one batch (GP and UPN; cone beam, parallel
  beam about z and the 3D parallel beam over the sphere; one with a stored
  A^T): after 25 iterations every problem has the oracle's gradient and
  function evaluation counts and final L, and its iterate is within 1e-9
  of the oracle's (relative to the largest voxel).
* FP32 with FP64 reductions at the batch workload's own tolerance (1e-6
  relative gradient map): two of its 32 problems, solved in a batch of
  three, against the oracle's UPN minimiser x* at 1e-8 (stored by
  tests/golden/make_batch_xstar.py).  Both sides read b rounded to FP32.
  The distance at 1e-6 is the tolerance's, not the precision's (a 1e-6
  relative gradient map leaves an objective gap of order 1e-4 on these
  problems), so the FP32 result must be within max(3 x the FP64 batch's own
  distance, 1e-5) relative L2 of x*, and the oracle's objective at it above
  phi* by at most 3 x the FP64 result's gap.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")
DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        DEV, torch.float64 if prec == tv.F64 else torch.float32)


def step_problems():
    """(geometry, phantom seed, method pair, alpha, stored A^T)"""
    return [
        (synth.cone_geometry(16, 7, 24, 20, 1.5, 64.0, 96.0), 21, (tv.UPN, oracle.UPN), 1e-2,
         False),
        (synth.Geometry(19, 13, 11, synth.view_angles(5, np.pi), synth.PARALLEL, 27, 14, 1.0,
                        1.0), 22, (tv.GP, oracle.GP), 3e-3, False),
        (synth.parallel3d_geometry(12, synth.sphere_directions(9), 18, 18, 1.2), 23,
         (tv.UPN, oracle.UPN), 1e-2, False),
        (synth.cone_geometry(24, 11, 36, 30, 1.5, 96.0, 144.0), 24, (tv.UPN, oracle.UPN), 1e-3,
         True),
        (synth.cone_geometry(10, 4, 16, 12, 1.5, 40.0, 60.0), 25, (tv.GP, oracle.GP), 1e-2,
         True),
    ]


def test_batched_fp64_takes_the_oracles_steps():
    K = 25
    geoms, bs, params, refs = [], [], [], []
    for i, (geom, seed, (mt, mo), alpha, stored) in enumerate(step_problems()):
        og = oracle.Geometry(geom)
        n = geom.nx
        x_true = synth.ellipsoid_phantom(n, 4, seed) if geom.nx == geom.ny == geom.nz else \
            synth.random_volume(og.vol_shape, seed)
        b = oracle.noisy_data(og, x_true, synth.unit_noise(og.proj_shape, seed + 50), 0.01)
        xo, io, _ = oracle.solve(og, b, method=mo, alpha=alpha, tau=1e-4, eps=0.0, max_iter=K,
                                 bt_form=1)
        refs.append((xo, io))
        G = tv.Geometry(geom, tv.F64)
        if stored:
            G.attach_matrix()
        geoms.append(G)
        bs.append(dev(b, tv.F64))
        params.append(dict(method=mt, alpha=alpha, tau=1e-4, eps=0.0, max_iter=K))
    print("batched fp64 vs oracle: 5 problems, 25 steps", flush=True)
    xs, infos, status = tv.solve_batched(geoms, bs, params)
    assert status == tv.ENOTCONV
    for i, (x, info, (xo, io)) in enumerate(zip(xs, infos, refs)):
        assert info["iters"] == io["iters"] == K, i
        assert (info["grad_evals"], info["func_evals"]) == (io["grad_evals"], io["func_evals"]), i
        assert info["L"] == io["L"], i
        err = np.max(np.abs(x.cpu().numpy() - xo)) / np.max(np.abs(xo))
        print(f"  problem {i}: max err {err:.2e}", flush=True)
        assert err <= 1e-9, (i, err)
        assert info["phi"] == pytest.approx(io["phi"], rel=1e-11)


def batch_xstar():
    meta = json.load(open(os.path.join(GOLDEN, "batch_xstar.json")))
    ws = synth.cfg_batch()
    out = []
    for key, m in sorted(meta.items()):
        p = int(key)
        w = ws[p]
        xs = np.load(os.path.join(GOLDEN, f"batch_xstar_p{p}.npy")).astype(np.float64)
        out.append((p, w, xs, m))
    return out


def test_batched_fp32_at_workload_tolerance_reaches_oracle_minimiser():
    cases = batch_xstar()
    ws = synth.cfg_batch()
    extra = 26  # a third, larger problem in the same batch (48^3, 14 views)
    members = [(p, ws[p]) for p, _, _, _ in cases] + [(extra, ws[extra])]
    data = []
    for p, w in members:
        og = oracle.Geometry(w.geom)
        b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
        data.append(np.asarray(b, np.float32).astype(np.float64))  # b rounded to FP32
    res = {}
    for prec in (tv.F32, tv.F64):
        geoms = [tv.Geometry(w.geom, prec) for _, w in members]
        bs = [dev(b, prec) for b in data]
        params = [dict(method=tv.UPN, alpha=w.alpha, tau=w.tau, eps=1e-6, max_iter=10000)
                  for _, w in members]
        print(f"batch of 3 workload problems to 1e-6, prec {prec}", flush=True)
        xs, infos, status = tv.solve_batched(geoms, bs, params)
        assert status == tv.OK, [i["stop_reason"] for i in infos]
        res[prec] = ([x.cpu().double().numpy() for x in xs], infos)
    for j, (p, w, x_star, m) in enumerate(cases):
        og = oracle.Geometry(w.geom)
        x32, x64 = res[tv.F32][0][j], res[tv.F64][0][j]
        d32 = np.linalg.norm(x32 - x_star) / np.linalg.norm(x_star)
        d64 = np.linalg.norm(x64 - x_star) / np.linalg.norm(x_star)
        ma32 = np.max(np.abs(x32 - x_star))
        phi32 = oracle.phi(og, data[j], w.alpha, w.tau, x32)
        phi64 = oracle.phi(og, data[j], w.alpha, w.tau, x64)
        gap32, gap64 = (phi32 - m["phi"]) / m["phi"], (phi64 - m["phi"]) / m["phi"]
        print(f"  problem {p} ({w.name}): FP32 rel-L2 {d32:.3e} max-abs {ma32:.3e} phi gap "
              f"{gap32:.3e}; FP64 rel-L2 {d64:.3e} phi gap {gap64:.3e}", flush=True)
        assert d32 <= max(3.0 * d64, 1e-5)
        assert -1e-10 <= gap32 <= max(3.0 * gap64, 1e-9)
        assert x32.min() >= 0.0
