"""Seeded random small scans of all three beams (parallel about z, cone,
parallel along directions over the sphere) with ragged volume and detector
sizes, arbitrary pitches, angles and directions: the projector, the on-the-fly
backprojector and the stored A^T against the FP64 oracle.  FP64: within 1e-12
of the output scale.  FP32 storage: the oracle is applied to the same
FP32-rounded inputs, and each output may differ by 2^-24 of (|ref| + the
oracle applied to the absolute input: the rounding of each stored length and
of the output) plus 1e-9 of the scale for the FP64 accumulation order.  The
stored transpose's non-zero count equals the oracle's up to the
coincident-crossing slivers."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")


def random_geometry(seed):
    rng = np.random.default_rng(1000 + seed)
    nx, ny, nz = (int(v) for v in rng.integers(3, 21, 3))
    V = int(rng.integers(1, 8))
    cols, rows = (int(v) for v in rng.integers(2, 26, 2))
    pu, pv = (float(v) for v in rng.uniform(0.7, 2.3, 2))
    beam = seed % 3
    if beam == 0:
        return synth.Geometry(nx, ny, nz, rng.uniform(0, math.pi, V), synth.PARALLEL, cols, rows,
                              pu, pv)
    if beam == 1:
        half = 0.5 * math.sqrt(nx * nx + ny * ny + nz * nz)
        R = half * rng.uniform(1.2, 4.0)
        SDD = R + half * rng.uniform(1.2, 4.0)
        return synth.Geometry(nx, ny, nz, rng.uniform(0, 2 * math.pi, V), synth.CONE, cols, rows,
                              pu, pv, R, SDD)
    d = rng.standard_normal((V, 3)) * rng.uniform(0.3, 3.0, (V, 1))
    return synth.Geometry(nx, ny, nz, np.zeros(V), synth.PARALLEL3D, cols, rows, pu, pv,
                          dirs=d)


def close(got, ref, absref, prec):
    scale = max(np.max(np.abs(ref)), 1e-300)
    if prec == tv.F64:
        return np.max(np.abs(got - ref)) <= 1e-12 * scale
    return bool(np.all(np.abs(got - ref) <= 2.0 ** -24 * (absref + np.abs(ref)) + 1e-9 * scale))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("seed", range(24))
def test_random_geometry_operators_match_oracle(seed, prec):
    g = random_geometry(seed)
    print(f"seed {seed} {prec}: beam {g.beam}, volume {g.nx}x{g.ny}x{g.nz}, {g.n_views} views, "
          f"detector {g.det_cols}x{g.det_rows}", flush=True)
    P = tv.F64 if prec == "f64" else tv.F32
    dt = torch.float64 if prec == "f64" else torch.float32
    rng = np.random.default_rng(2000 + seed)
    x = rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx))
    r = rng.standard_normal(g.proj_shape)
    if prec == "f32":  # the oracle sees the same rounded inputs
        x, r = x.astype(np.float32).astype(np.float64), r.astype(np.float32).astype(np.float64)
    G = tv.Geometry(g, P)
    xd = torch.from_numpy(x).to("cuda", dt)
    rd = torch.from_numpy(r).to("cuda", dt)
    y_ref, b_ref = oracle.project(g, x), oracle.backproject(g, r)
    b_abs = oracle.backproject(g, np.abs(r))
    assert close(tv.project(G, xd).cpu().double().numpy(), y_ref, y_ref, P)
    assert close(tv.backproject(G, rd).cpu().double().numpy(), b_ref, b_abs, P)
    nnz = G.attach_matrix()
    ref_nnz = oracle.nnz(g)
    assert abs(nnz - ref_nnz) <= 4e-6 * ref_nnz + 16, (nnz, ref_nnz)
    assert close(tv.backproject(G, rd).cpu().double().numpy(), b_ref, b_abs, P)


@pytest.mark.parametrize("stored", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_random_geometry_upn_steps_match_oracle_fp64(seed, stored):
    """25 UPN steps (FP64) on a random scan take the oracle's steps: the same
    line-search L sequence and iterates within 1e-9 of their scale, with the
    backprojection on the fly or from the stored A^T."""
    g = random_geometry(seed)
    print(f"seed {seed} stored={stored}: UPN steps, beam {g.beam}, volume {g.nx}x{g.ny}x{g.nz}",
          flush=True)
    rng = np.random.default_rng(3000 + seed)
    og = oracle.Geometry(g)
    x_true = rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx))
    b = oracle.noisy_data(og, x_true, rng.standard_normal(g.proj_shape), 0.01)
    K, alpha, tau = 25, 1e-2, 1e-2
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=alpha, tau=tau, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(g, tv.F64)
    if stored:
        G.attach_matrix()
    x, info, h = tv.solve(G, torch.from_numpy(b).to("cuda", torch.float64), method=tv.UPN,
                          alpha=alpha, tau=tau, eps=0.0, max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"] == K
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    err = np.max(np.abs(x.cpu().numpy() - xo)) / max(np.max(np.abs(xo)), 1e-300)
    assert err <= 1e-9, err


def test_random_geometries_batched_equals_single_fp32():
    """Five random scans (every beam; some with a stored A^T) solved together
    equal their single solves bit for bit: the grouped kernels run the single
    kernels' block bodies with the same block decomposition."""
    seeds = [0, 1, 2, 4, 5]
    geoms, bs, params = [], [], []
    for q, seed in enumerate(seeds):
        g = random_geometry(seed)
        rng = np.random.default_rng(4000 + seed)
        og = oracle.Geometry(g)
        b = oracle.noisy_data(og, rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx)),
                              rng.standard_normal(g.proj_shape), 0.01)
        G = tv.Geometry(g, tv.F32)
        if q % 2:
            G.attach_matrix()
        geoms.append(G)
        bs.append(torch.from_numpy(b).to("cuda", torch.float32))
        params.append(dict(method=tv.UPN if q % 3 else tv.GP, alpha=10.0 ** -(1 + q % 3),
                           tau=1e-2, eps=1e-4, max_iter=150))
    print(f"batched vs single: seeds {seeds}", flush=True)
    singles = [tv.solve(G, b, **p) for G, b, p in zip(geoms, bs, params)]
    xb, ib, _ = tv.solve_batched(geoms, bs, params)
    for i, (x, info, _) in enumerate(singles):
        assert torch.equal(xb[i], x), i
        assert ib[i]["iters"] == info["iters"], i


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_geometry_unrolled_matches_oracle_fp64(seed):
    """The differentiated form on a random scan of each beam (FP64, K = 10):
    the oracle's L sequence, x_K within 1e-10, and dl/dlog(alpha), dl/db
    within 1e-8 of the oracle's reverse pass for l = |x_K - x_true|^2."""
    g = random_geometry(seed)
    print(f"seed {seed}: unrolled, beam {g.beam}, volume {g.nx}x{g.ny}x{g.nz}", flush=True)
    rng = np.random.default_rng(5000 + seed)
    og = oracle.Geometry(g)
    xt = rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx))
    b = oracle.noisy_data(og, xt, rng.standard_normal(g.proj_shape), 0.01)
    K, alpha, tau = 10, 1e-2, 1e-2
    o = oracle.unrolled(og, b, K, alpha, tau=tau)
    og_g = oracle.unrolled(og, b, K, alpha, tau=tau, L=o["L"], xK_bar=2.0 * (o["xK"] - xt))
    G = tv.Geometry(g, tv.F64)
    bd = torch.from_numpy(b).to("cuda", torch.float64)
    xK, tape, L = tv.upn_unrolled_fwd(G, bd, K, alpha, tau=tau)
    np.testing.assert_array_equal(np.array(L), o["L"])
    xk = xK.cpu().numpy()
    assert np.linalg.norm(xk - o["xK"]) <= 1e-10 * np.linalg.norm(o["xK"])
    da, db = tv.upn_unrolled_bwd(G, bd, tape, 2.0 * (xK - torch.from_numpy(xt).to("cuda")))
    ref = alpha * og_g["alpha_bar"]
    assert abs(da - ref) <= 1e-8 * abs(ref)
    assert np.linalg.norm(db.cpu().numpy() - og_g["b_bar"]) <= 1e-8 * np.linalg.norm(og_g["b_bar"])


@pytest.mark.parametrize("method", ["gp", "upn"])
@pytest.mark.parametrize("seed", [3, 4, 5])
def test_random_geometry_box_steps_match_oracle_fp64(seed, method):
    """25 steps of GP or UPN under the box Q = [0.05, 0.8]^N (FP64) on a
    random scan: the oracle's L sequence, iterates within 1e-9, all in Q."""
    lo, hi = 0.05, 0.8
    g = random_geometry(seed)
    print(f"seed {seed}: {method} in a box, beam {g.beam}", flush=True)
    rng = np.random.default_rng(6000 + seed)
    og = oracle.Geometry(g)
    b = oracle.noisy_data(og, rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx)),
                          rng.standard_normal(g.proj_shape), 0.01)
    tm, om = (tv.GP, oracle.GP) if method == "gp" else (tv.UPN, oracle.UPN)
    K, alpha, tau = 25, 1e-2, 1e-2
    xo, io, ho = oracle.solve(og, b, method=om, alpha=alpha, tau=tau, eps=0.0, max_iter=K,
                              hist_len=K, bt_form=1, lower=lo, upper=hi)
    G = tv.Geometry(g, tv.F64)
    x, info, h = tv.solve(G, torch.from_numpy(b).to("cuda", torch.float64), method=tm,
                          alpha=alpha, tau=tau, eps=0.0, max_iter=K, hist_len=K, lower=lo,
                          upper=hi)
    assert info["iters"] == io["iters"]
    n = len(h["L"])
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:n])
    xg = x.cpu().numpy()
    assert xg.min() >= lo and xg.max() <= hi
    assert np.max(np.abs(xg - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)
