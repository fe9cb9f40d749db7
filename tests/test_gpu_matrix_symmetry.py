"""The stored transpose in its symmetric layout (one cell of the scan's
symmetry group stored, every entry applied to all images of its voxel).

* The layout is chosen only where the scan has the symmetry: quarter turns
  (V divisible by 4, square even volume), half turns (V even, ny even) and
  the z mirror (nz even), with an even detector; otherwise fewer images or
  the plain layout.  tvreg_matrix_symmetry reports the number of voxels one
  entry serves, and the matrix shrinks by about that factor.
* Products from it match the oracle: FP64 within 1e-12 of the output scale,
  FP32 within the rounding of the stored values and of the output; and they
  match the plain layout's products within 1e-13 (FP64: the images' lengths
  differ from the directly computed ones only by the rounding of the view
  angles' cosines).
* The FP64 solver takes the oracle's steps with it.
* The solvers' projection through the companion copy equals the plain
  projection bit for bit (and so the oracle's).
* The on-the-fly backprojector gathers through the same symmetry (no stored
  transpose): its products match the oracle at the operator bar and the
  plain gather within 1e-13 of the output scale, and on the cell the images
  tile the volume from (the identity image) they are the plain gather's own
  sums, bit for bit.  The solver takes the oracle's steps with it too.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from test_gpu_operators import rounded, to_dev

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")


def cone(nx, ny, nz, angles, cols, rows, pitch=1.5, R=None, SDD=None):
    n = max(nx, ny, nz)
    R = 4.0 * n if R is None else R
    SDD = 6.0 * n if SDD is None else SDD
    return synth.Geometry(nx, ny, nz, np.asarray(angles, np.float64), synth.CONE, cols, rows,
                          pitch, pitch, R, SDD)


def full_circle(V, offset=0.0):
    return offset + synth.view_angles(V, 2 * math.pi)


PERTURBED = full_circle(8)
PERTURBED[3] += 1e-6

# name: (geometry, expected voxels per stored entry)
CASES = {
    "quarter_mirror": (cone(12, 12, 12, full_circle(8), 18, 16), 8),
    "quarter_mirror_offset": (cone(12, 12, 12, full_circle(12, 0.3), 18, 16), 8),
    "quarter_odd_nz": (cone(12, 12, 9, full_circle(8), 18, 14), 4),
    "half_mirror": (cone(9, 10, 8, full_circle(6), 16, 14), 4),
    "half_odd_nz": (cone(11, 16, 7, full_circle(10), 16, 12), 2),
    "mirror_only": (cone(7, 9, 10, full_circle(5), 14, 16), 2),
    # an odd row count puts the w = 0 row exactly in the z = 0 voxel face
    # (well posed, half-open cells): no symmetric layout.  (An odd column
    # count would also put the u = 0 column in a face at theta = pi / 2, where
    # cos is 6e-17 and the ray's cells are ill-posed for any two codes.)
    "odd_rows": (cone(12, 12, 12, full_circle(8), 18, 17), 1),
    "perturbed_angles": (cone(12, 12, 12, PERTURBED, 18, 16), 2),
    "cone64": (synth.cfg_cone64().geom, 8),
}


def host(t):
    return t.detach().cpu().double().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_symmetry_order_and_size(name):
    g, order = CASES[name]
    print(f"symmetry {name}", flush=True)
    G = tv.Geometry(g, tv.F32)
    nnz = G.attach_matrix()
    assert G.symmetry == order
    size_sym = G.matrix_bytes
    P = tv.Geometry(g, tv.F32)
    nnz_plain = P.attach_matrix(symmetric=False)
    assert P.symmetry == 1
    # every stored entry stands for `order` entries of A; the few sub-ulp
    # segments coincident crossings leave (lengths ~1e-16) are counted once
    # per image, so their count scales with the order
    assert abs(nnz - nnz_plain) <= 4e-6 * nnz_plain + 16 * order
    if order > 1:
        assert size_sym < 1.6 * P.matrix_bytes / order


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("name", list(CASES))
def test_symmetric_product_matches_oracle(name, prec):
    g, order = CASES[name]
    print(f"symmetric A^T {name} prec={prec}", flush=True)
    G = tv.Geometry(g, prec)
    G.attach_matrix()
    assert G.symmetry == order
    r = rounded(np.random.default_rng(51).standard_normal(g.proj_shape), prec)
    got = host(tv.backproject(G, to_dev(r, prec)))
    ref = oracle.backproject(g, r)
    scale = max(np.max(np.abs(ref)), 1e-300)
    if prec == tv.F64:
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
        P = tv.Geometry(g, prec)
        P.attach_matrix(symmetric=False)
        plain = host(tv.backproject(P, to_dev(r, prec)))
        assert np.max(np.abs(got - plain)) <= 1e-13 * scale
    else:
        bound = oracle.backproject(g, np.abs(r))
        tol = 2.0 ** -24 * (bound + np.abs(ref)) + 1e-9 * scale
        bad = np.abs(got - ref) > tol
        assert not bad.any(), f"{bad.sum()} entries off"


@pytest.mark.parametrize("name", ["quarter_mirror", "half_mirror", "mirror_only"])
def test_symmetric_adjoint_identity_fp64(name):
    g, _ = CASES[name]
    G = tv.Geometry(g, tv.F64)
    G.attach_matrix()
    rng = np.random.default_rng(52)
    x = to_dev(rng.standard_normal(g.vol_shape), tv.F64)
    r = to_dev(rng.standard_normal(g.proj_shape), tv.F64)
    lhs = float(torch.sum(tv.project(G, x) * r))
    rhs = float(torch.sum(x * tv.backproject(G, r)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_symmetric_solver_first_iterations_match_oracle_fp64():
    g, _ = CASES["quarter_mirror"]
    og = oracle.Geometry(g)
    b = oracle.noisy_data(og, synth.ellipsoid_phantom(12, 4, 53),
                          synth.unit_noise(og.proj_shape, 54), 0.01)
    K = 25
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(g, tv.F64)
    G.attach_matrix()
    assert G.symmetry == 8
    x, info, h = tv.solve(G, to_dev(b, tv.F64), method=tv.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                          max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"]
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    assert np.max(np.abs(host(x) - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)


def test_symmetry_switch_needs_detached_matrix():
    g, _ = CASES["quarter_mirror"]
    G = tv.Geometry(g, tv.F32)
    G.attach_matrix()
    with pytest.raises(tv.TvregError) as e:
        tv._check(tv.lib().tvreg_set_symmetry(G.handle, 0), "set_symmetry")
    assert e.value.status == tv.EINVAL
    G.detach_matrix()
    tv._check(tv.lib().tvreg_set_symmetry(G.handle, 0), "set_symmetry")
    assert tv.lib().tvreg_matrix_symmetry(G.handle) == 1
    tv._check(tv.lib().tvreg_set_symmetry(G.handle, 1), "set_symmetry")
    assert tv.lib().tvreg_matrix_symmetry(G.handle) == 8


# the group of each case: (turns, mirror)
GROUPS = {"quarter_mirror": (4, 1), "quarter_mirror_offset": (4, 1), "quarter_odd_nz": (4, 0),
          "half_mirror": (2, 1), "half_odd_nz": (2, 0), "mirror_only": (1, 1), "odd_rows": (1, 0),
          "perturbed_angles": (1, 1), "cone64": (4, 1)}


def rot_mir_order(name):
    rot, mir = GROUPS[name]
    return rot * (2 if mir else 1)


def cell_of(name, g):
    """The cell the images tile the volume from (the identity image): x <
    nx / 2 and y < ny / 2 for quarter turns, y < ny / 2 for half turns,
    z < nz / 2 with the mirror."""
    rot, mir = GROUPS[name]
    return (slice(0, g.nz // 2 if mir else g.nz), slice(0, g.ny // 2 if rot >= 2 else g.ny),
            slice(0, g.nx // 2 if rot == 4 else g.nx))


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("name", list(CASES))
def test_symmetric_gather_matches_oracle(name, prec):
    g, order = CASES[name]
    print(f"symmetric gather {name} prec={prec}", flush=True)
    G = tv.Geometry(g, prec)
    r = rounded(np.random.default_rng(61).standard_normal(g.proj_shape), prec)
    got = host(tv.backproject(G, to_dev(r, prec)))
    ref = oracle.backproject(g, r)
    scale = max(np.max(np.abs(ref)), 1e-300)
    if prec == tv.F64:
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
        P = tv.Geometry(g, prec)
        P.set_symmetry(False)
        plain = host(tv.backproject(P, to_dev(r, prec)))
        assert np.max(np.abs(got - plain)) <= 1e-13 * scale
        assert rot_mir_order(name) == order
        c = cell_of(name, g)
        np.testing.assert_array_equal(got[c], plain[c])
    else:
        bound = oracle.backproject(g, np.abs(r))
        tol = 2.0 ** -24 * (bound + np.abs(ref)) + 1e-9 * scale
        bad = np.abs(got - ref) > tol
        assert not bad.any(), f"{bad.sum()} entries off"


@pytest.mark.parametrize("name", ["quarter_mirror", "half_odd_nz", "mirror_only"])
def test_symmetric_gather_adjoint_identity_fp64(name):
    g, _ = CASES[name]
    G = tv.Geometry(g, tv.F64)
    rng = np.random.default_rng(62)
    x = to_dev(rng.standard_normal(g.vol_shape), tv.F64)
    r = to_dev(rng.standard_normal(g.proj_shape), tv.F64)
    lhs = float(torch.sum(tv.project(G, x) * r))
    rhs = float(torch.sum(x * tv.backproject(G, r)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_symmetric_gather_solver_first_iterations_match_oracle_fp64():
    g, _ = CASES["half_mirror"]
    og = oracle.Geometry(g)
    b = oracle.noisy_data(og, synth.random_volume(g.vol_shape, 63),
                          synth.unit_noise(og.proj_shape, 64), 0.01)
    K = 25
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(g, tv.F64)
    assert tv.lib().tvreg_matrix_symmetry(G.handle) == 4  # the group the gather uses
    x, info, h = tv.solve(G, to_dev(b, tv.F64), method=tv.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                          max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"]
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    assert np.max(np.abs(host(x) - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)



@pytest.mark.parametrize("cols", [1, 2, 64])
@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("name", ["quarter_mirror", "half_odd_nz", "mirror_only", "odd_rows"])
def test_companion_projection_matches_plain_and_oracle(name, prec, cols):
    """The solvers' projection (tvreg_project_ws: the companion copy of the
    tile) is tvreg_project's bit for bit, and the oracle's at the operator
    bar."""
    g, _ = CASES[name]
    print(f"companion projection {name} prec={prec} cols={cols}", flush=True)
    G = tv.Geometry(g, prec)
    G.set_tuning(cols, 4, 8)
    x = rounded(synth.random_volume(g.vol_shape, 65), prec)
    got = host(tv.project(G, to_dev(x, prec), workspace=tv.project_workspace(G)))
    np.testing.assert_array_equal(got, host(tv.project(G, to_dev(x, prec))))
    ref = oracle.project(g, x)
    scale = max(np.max(np.abs(ref)), 1e-300)
    if prec == tv.F64:
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
    else:
        tol = 2.0 ** -24 * np.abs(ref) + 1e-9 * scale
        assert not (np.abs(got - ref) > tol).any()


def test_project_ws_rejects_short_workspace():
    g, _ = CASES["quarter_mirror"]
    G = tv.Geometry(g, tv.F32)
    x = to_dev(np.zeros(g.vol_shape), tv.F32)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(tv.TvregError) as e:
        tv.project(G, x, workspace=ws)
    assert e.value.status == tv.ENOMEM


@pytest.mark.parametrize("name", ["quarter_mirror", "half_mirror", "mirror_only"])
def test_column_tile_solver_first_iterations_match_oracle_fp64(name):
    """25 UPN steps with column tiles (z-fastest companion) and the symmetric
    gather take the oracle's steps."""
    g, _ = CASES[name]
    og = oracle.Geometry(g)
    b = oracle.noisy_data(og, synth.random_volume(g.vol_shape, 66),
                          synth.unit_noise(og.proj_shape, 67), 0.01)
    K = 25
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    G = tv.Geometry(g, tv.F64)
    G.set_tuning(2, 4, 8)
    x, info, h = tv.solve(G, to_dev(b, tv.F64), method=tv.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                          max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"]
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    assert np.max(np.abs(host(x) - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)
