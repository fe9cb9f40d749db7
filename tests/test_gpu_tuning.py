"""Tile-shape tuning of the on-the-fly operators (tvreg_autotune,
tvreg_set_tuning).

* Every projector shape (ray tiles of 1 x 64, 2 x 32 (column tiles), 8 x 8,
  16 x 4, 32 x 2, 64 x 1 pixels per wave; 1, 2, 4, 8 waves per block) and
  every backprojector depth (4, 8, 16 voxels per thread along z) gives
  bitwise the same outputs as the defaults, and those match the oracle (the
  operator parity tests' bar), on every test geometry and both precisions.
* The default ray tile follows the detector's row count (2 columns for a
  multiple of 32 rows, else 64).
* The tuner returns a listed shape with positive timings and keeps it.
* A solve under other shapes, column tiles (with their z-fastest companion
  copy) among them, still matches the oracle's iterations.
* The batched solve gives the same result under any of the geometry's
  shapes (it runs each problem with its own, depth 16 at 8).
* Out-of-list shapes are rejected.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from test_gpu_operators import GEOMS, check_close, rounded, to_dev

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")


def default_tuning(g):
    """The documented default shapes for a geometry."""
    rows = g.det_rows
    return (2 if rows % 32 == 0 else 64, 4, 8)


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("name", list(GEOMS))
def test_every_shape_gives_identical_operators(name, prec):
    print(f"shapes {name} prec={prec}", flush=True)
    g = GEOMS[name]
    G = tv.Geometry(g, prec)
    assert G.tuning == default_tuning(g)
    rng = np.random.default_rng(51)
    x = rounded(rng.uniform(0.0, 1.0, (g.nz, g.ny, g.nx)), prec)
    r = rounded(rng.standard_normal(g.proj_shape), prec)
    xd, rd = to_dev(x, prec), to_dev(r, prec)
    y0, b0 = tv.project(G, xd), tv.backproject(G, rd)
    check_close(y0, oracle.project(g, x), prec, f"A x [{name}]")
    if prec == tv.F64:
        check_close(b0, oracle.backproject(g, r), prec, f"A^T r [{name}]")
    for cols in tv.PROJECT_TILE_COLS:
        for waves in tv.PROJECT_WAVES:
            G.set_tuning(cols, waves, 8)
            assert G.tuning == (cols, waves, 8)
            assert torch.equal(tv.project(G, xd), y0), (cols, waves)
    for depth in tv.BACKPROJECT_DEPTHS:
        G.set_tuning(64, 4, depth)
        assert torch.equal(tv.backproject(G, rd), b0), depth


@pytest.mark.parametrize("prec", [tv.F32, tv.F64])
def test_autotune_picks_a_listed_shape(prec):
    g = GEOMS["cone64"]
    G = tv.Geometry(g, prec)
    t = G.autotune(reps=3)
    print(f"autotune cone64 prec={prec}: {t}", flush=True)
    assert t["project_tile_cols"] in tv.PROJECT_TILE_COLS
    assert t["project_waves"] in tv.PROJECT_WAVES
    assert t["backproject_depth"] in tv.BACKPROJECT_DEPTHS
    assert len(t["project_ms"]) == 24 and all(v > 0 for v in t["project_ms"].values())
    assert all(v > 0 for v in t["backproject_ms"].values())
    chosen = (t["project_tile_cols"], t["project_waves"])
    assert t["project_ms"][chosen] == min(t["project_ms"].values())
    assert t["backproject_ms"][t["backproject_depth"]] == min(t["backproject_ms"].values())
    assert G.tuning == chosen + (t["backproject_depth"],)
    x = to_dev(np.random.default_rng(52).uniform(0, 1, (g.nz, g.ny, g.nx)), prec)
    assert torch.equal(tv.project(G, x), tv.project(tv.Geometry(g, prec), x))


def test_autotune_with_stored_matrix_times_on_the_fly_shapes():
    g = GEOMS["cone_ragged"]
    G = tv.Geometry(g, tv.F64)
    G.attach_matrix()
    r = to_dev(np.random.default_rng(53).standard_normal(g.proj_shape), tv.F64)
    before = tv.backproject(G, r)
    t = G.autotune(reps=2)
    assert t["backproject_depth"] in tv.BACKPROJECT_DEPTHS
    assert torch.equal(tv.backproject(G, r), before)  # still the stored product


@pytest.mark.parametrize("shape", [(8, 1, 16), (16, 8, 4), (32, 2, 8), (1, 4, 8), (2, 1, 4),
                                   (64, 4, 8)])
def test_solve_under_other_shapes_matches_oracle_fp64(shape):
    w = synth.cfg_small_parallel()
    og = oracle.Geometry(w.geom)
    b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
    K = 25
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(w.geom, tv.F64)
    G.set_tuning(*shape)
    x, info, h = tv.solve(G, to_dev(b, tv.F64), method=tv.UPN, alpha=w.alpha, tau=w.tau,
                          eps=0.0, max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"]
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    xh = x.cpu().numpy()
    assert np.max(np.abs(xh - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)


def test_batched_solve_same_under_any_tuning():
    w = synth.cfg_small_parallel()
    og = oracle.Geometry(w.geom)
    b = to_dev(oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta), tv.F32)
    p = dict(alpha=w.alpha, tau=w.tau, eps=1e-4, max_iter=150)
    G0 = tv.Geometry(w.geom, tv.F32)
    x0, i0, _ = tv.solve_batched([G0], [b], [p])
    G = tv.Geometry(w.geom, tv.F32)
    G.set_tuning(8, 1, 16)
    x1, i1, _ = tv.solve_batched([G], [b], [p])
    assert torch.equal(x1[0], x0[0])
    assert i1[0]["iters"] == i0[0]["iters"]
    assert G.tuning == (8, 1, 16)


@pytest.mark.parametrize("shape", [(64, 3, 8), (64, 0, 8), (64, 16, 8), (64, 4, 2),
                                   (64, 4, 32), (64, 4, -8), (4, 4, 8), (128, 4, 8),
                                   (48, 4, 8), (0, 4, 8)])
def test_set_tuning_rejects_unlisted_shapes(shape):
    G = tv.Geometry(GEOMS["cone8"], tv.F32)
    with pytest.raises(tv.TvregError, match="must be"):
        G.set_tuning(*shape)
    assert G.tuning == default_tuning(GEOMS["cone8"])


def test_autotune_rejects_bad_reps():
    G = tv.Geometry(GEOMS["cone8"], tv.F32)
    with pytest.raises(tv.TvregError, match="reps"):
        G.autotune(reps=0)
