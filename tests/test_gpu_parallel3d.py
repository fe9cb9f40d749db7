"""GPU parity of the 3D parallel beam (the paper's Sec. IV-A geometry: view
directions over the unit sphere) against the FP64 oracle.

* Projector (the walk on rays formed from each view's direction and detector
  axes) and the voxel-driven gather backprojector: FP64 within 1e-12 of the
  output scale; FP32 per element within its own rounding (the operator
  tests' bars); on ragged volumes, oblique, axis-aligned, downward and
  unnormalised directions, and at the paper's size (64^3, 55 views of 91^2).
* The stored A^T: non-zero count = the oracle's (up to the coincident-
  crossing slivers), products and the adjoint identity; on-the-fly and
  stored transposes agree.
* Every tile shape gives bitwise the same operators.
* UPN in FP64 takes the oracle's steps (same L sequence, iterates within
  1e-9); the batched solve equals the single solve bit for bit.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from test_gpu_operators import check_close, rounded, to_dev

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")


def g3(nx, ny, nz, dirs, cols, rows, pitch=1.0):
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    return synth.Geometry(nx, ny, nz, np.zeros(len(d)), synth.PARALLEL3D, cols, rows, pitch,
                          pitch, dirs=d)


GEOMS3 = {
    "ragged_oblique": g3(13, 11, 9, np.vstack([synth.sphere_directions(5),
                                               [[0.3, -0.8, -0.52], [-2.0, 0.5, 1.0]]]),
                         17, 14, 1.1),
    "axes": g3(6, 7, 5, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0], [0, -3, 0]], 8, 8),
    "in_plane": g3(9, 9, 6, [[math.cos(t), math.sin(t), 0.0] for t in (0.2, 1.3, 2.6)], 12,
                   8),
    "paper_small": synth.parallel3d_geometry(16, synth.sphere_directions(9), 23, 23,
                                             math.sqrt(3.0) * 16 / 23),
}


def data3(g, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx)), rng.standard_normal(g.proj_shape)


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("name", list(GEOMS3))
def test_3d_operators_match_oracle(name, prec):
    print(f"3d operators {name} prec={prec}", flush=True)
    g = GEOMS3[name]
    G = tv.Geometry(g, prec)
    x, r = data3(g, 61)
    x, r = rounded(x, prec), rounded(r, prec)
    check_close(tv.project(G, to_dev(x, prec)), oracle.project(g, x), prec, f"A x [{name}]")
    got = tv.backproject(G, to_dev(r, prec)).cpu().double().numpy()
    ref = oracle.backproject(g, r)
    scale = np.max(np.abs(ref))
    if prec == tv.F64:
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
    else:
        bound = oracle.backproject(g, np.abs(r))
        assert np.all(np.abs(got - ref) <= 2.0 ** -24 * (bound + np.abs(ref)) + 1e-9 * scale)


@pytest.mark.parametrize("name", list(GEOMS3))
def test_3d_stored_transpose(name):
    g = GEOMS3[name]
    G0 = tv.Geometry(g, tv.F64)
    G = tv.Geometry(g, tv.F64)
    nnz = G.attach_matrix()
    ref_nnz = oracle.nnz(g)
    assert abs(nnz - ref_nnz) <= 4e-6 * ref_nnz + 16, (nnz, ref_nnz)
    x, r = data3(g, 62)
    xd, rd = to_dev(x, tv.F64), to_dev(r, tv.F64)
    atr, atr0 = tv.backproject(G, rd), tv.backproject(G0, rd)
    ref = oracle.backproject(g, r)
    assert np.max(np.abs(atr.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert float((atr - atr0).abs().max()) <= 1e-13 * float(atr0.abs().max())
    lhs = float(torch.sum(tv.project(G, xd) * rd))
    rhs = float(torch.sum(xd * atr))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
def test_3d_every_shape_identical(prec):
    g = GEOMS3["ragged_oblique"]
    G = tv.Geometry(g, prec)
    x, r = data3(g, 63)
    xd, rd = to_dev(rounded(x, prec), prec), to_dev(rounded(r, prec), prec)
    y0, b0 = tv.project(G, xd), tv.backproject(G, rd)
    for cols in tv.PROJECT_TILE_COLS:
        for waves in tv.PROJECT_WAVES:
            G.set_tuning(cols, waves, 8)
            assert torch.equal(tv.project(G, xd), y0), (cols, waves)
    for depth in tv.BACKPROJECT_DEPTHS:
        G.set_tuning(64, 4, depth)
        assert torch.equal(tv.backproject(G, rd), b0), depth


@pytest.fixture(scope="module")
def small_paper():
    g = GEOMS3["paper_small"]
    xt = synth.ellipsoid_phantom(16, 6, 71)
    b = oracle.noisy_data(g, xt, synth.unit_noise(g.proj_shape, 72), 0.01)
    return g, b


def test_3d_upn_steps_match_oracle_fp64(small_paper):
    g, b = small_paper
    K = 25
    xo, io, ho = oracle.solve(g, b, method=oracle.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(g, tv.F64)
    x, info, h = tv.solve(G, to_dev(b, tv.F64), method=tv.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                          max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"]
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    assert np.max(np.abs(x.cpu().numpy() - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)


def test_3d_batched_equals_single(small_paper):
    g, b = small_paper
    bd = to_dev(b, tv.F32)
    p = dict(alpha=1e-2, tau=1e-4, eps=1e-4, max_iter=300)
    Gs = [tv.Geometry(g, tv.F32), tv.Geometry(g, tv.F32)]
    Gs[1].attach_matrix()
    singles = [tv.solve(G, bd, method=tv.UPN, **p) for G in Gs]
    xb, ib, _ = tv.solve_batched(Gs, [bd, bd], [p, p])
    for i, (x, info, _) in enumerate(singles):
        assert torch.equal(xb[i], x), i
        assert ib[i]["iters"] == info["iters"], i


@pytest.mark.parametrize("views", [55, 19])
def test_3d_paper_size_operators(views):
    """The paper's geometry at full size (64^3, 91^2 pixels), FP32 storage:
    every output element within its own rounding of the oracle."""
    w = synth.cfg_paper(views)
    g = w.geom
    print(f"paper geometry, {views} views", flush=True)
    G = tv.Geometry(g, tv.F32)
    x = rounded(w.phantom(), tv.F32)
    check_close(tv.project(G, to_dev(x, tv.F32)), oracle.project(g, x), tv.F32,
                f"A x [paper {views}]")
    r = rounded(np.random.default_rng(64).standard_normal(g.proj_shape), tv.F32)
    ref = oracle.backproject(g, r)
    bound = oracle.backproject(g, np.abs(r))
    scale = np.max(np.abs(ref))
    for stored in (False, True):
        if stored:
            G.attach_matrix()
        got = tv.backproject(G, to_dev(r, tv.F32)).cpu().double().numpy()
        assert np.all(np.abs(got - ref) <= 2.0 ** -24 * (bound + np.abs(ref)) + 1e-9 * scale), \
            stored
