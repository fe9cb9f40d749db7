"""Pins of the oracle's 3D parallel beam (view directions over the unit
sphere, Sec. IV-A), each against something other than the oracle's own
formulas:

* directions in the x-y plane reproduce the parallel beam about z;
* the four axis directions +z, -z, +x, +y are column sums of the volume
  (the detector axes e_u = e_z x d / |.| or e_x, e_v = d x e_u fix which
  column and in which orientation);
* a volume of ones projects to each line's chord through the box, computed
  here with an independent slab intersection;
* Siddon lengths equal brute-force per-voxel slab lengths, and the
  backprojection is the adjoint, for oblique directions on a ragged volume.
"""
import math

import numpy as np

import oracle
import synth


def g3(nx, ny, nz, dirs, cols, rows, pitch=1.0):
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    return synth.Geometry(nx, ny, nz, np.zeros(len(d)), synth.PARALLEL3D, cols, rows, pitch,
                          pitch, dirs=d)


def test_in_plane_directions_reproduce_parallel_beam():
    th = np.array([0.3, 1.1, 2.0, 2.9])
    x = np.random.default_rng(1).uniform(0, 1, (5, 6, 7))
    g2 = synth.Geometry(7, 6, 5, th, synth.PARALLEL, 10, 8, 1.0, 1.0)
    d = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)
    y2, y3 = oracle.project(g2, x), oracle.project(g3(7, 6, 5, d, 10, 8), x)
    assert np.max(np.abs(y3 - y2)) <= 1e-12 * np.max(np.abs(y2))


def test_axis_directions_are_oriented_column_sums():
    n = 5
    x = np.random.default_rng(2).uniform(0, 1, (n, n, n))  # [z][y][x]
    g = g3(n, n, n, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0]], n, n)
    y = oracle.project(g, x)  # [view][row][col]
    # +z: e_u = e_x, e_v = e_y: (row, col) -> (iy, ix)
    np.testing.assert_allclose(y[0], x.sum(axis=0), rtol=0, atol=1e-12)
    # -z: e_u = e_x, e_v = -e_y: row runs against y
    np.testing.assert_allclose(y[1], x.sum(axis=0)[::-1, :], rtol=0, atol=1e-12)
    # +x: e_u = e_y, e_v = e_z: (row, col) -> (iz, iy)
    np.testing.assert_allclose(y[2], x.sum(axis=2), rtol=0, atol=1e-12)
    # +y: e_u = -e_x, e_v = e_z: (row, col) -> (iz, nx - 1 - ix)
    np.testing.assert_allclose(y[3], x.sum(axis=1)[:, ::-1], rtol=0, atol=1e-12)


def chord(S, d, half):
    """Length of the line S + t d (|d| = 1) inside the box [-half, half]."""
    lo, hi = -np.inf, np.inf
    for k in range(3):
        if d[k] == 0.0:
            if not (-half[k] <= S[k] <= half[k]):
                return 0.0
            continue
        a, b = (-half[k] - S[k]) / d[k], (half[k] - S[k]) / d[k]
        lo, hi = max(lo, min(a, b)), min(hi, max(a, b))
    return max(0.0, hi - lo)


def test_ones_project_to_chord_lengths():
    dirs = synth.sphere_directions(7) * np.array([1.0, 1.0, 1.0])
    dirs[3] = [0.3, -0.8, -0.52]  # not normalised, pointing down
    nx, ny, nz, cols, rows, pitch = 6, 5, 4, 9, 8, 1.1
    g = g3(nx, ny, nz, dirs, cols, rows, pitch)
    y = oracle.project(g, np.ones((nz, ny, nx)))
    half = np.array([nx, ny, nz]) / 2.0
    for v in range(len(dirs)):
        d = dirs[v] / np.linalg.norm(dirs[v])
        a = math.hypot(d[0], d[1])
        eu = np.array([-d[1] / a, d[0] / a, 0.0]) if a > 0 else np.array([1.0, 0.0, 0.0])
        ev = np.cross(d, eu)
        for row in range(rows):
            for col in range(cols):
                u = (col - (cols - 1) / 2) * pitch
                w = (row - (rows - 1) / 2) * pitch
                ref = chord(u * eu + w * ev, d, half)
                assert abs(y[v, row, col] - ref) <= 1e-12, (v, row, col, y[v, row, col], ref)


def test_siddon_matches_bruteforce_and_adjoint():
    dirs = np.vstack([synth.sphere_directions(5), [[0.2, 0.9, -0.4]]])
    g = g3(6, 5, 7, dirs, 8, 9, 0.9)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (7, 5, 6))
    y = oracle.project(g, x)
    yb = oracle.project_bruteforce(g, x)
    assert np.max(np.abs(y - yb)) <= 1e-13 * np.max(np.abs(yb))
    r = rng.standard_normal(y.shape)
    lhs, rhs = float(np.sum(y * r)), float(np.sum(x * oracle.backproject(g, r)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_sphere_directions_are_unit_and_spread():
    d = synth.sphere_directions(55)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(d[:, 2] > 0)
    # equal-area spiral: the smallest angle between two lines is not tiny
    c = np.abs(d @ d.T) - 2 * np.eye(len(d))
    assert math.degrees(math.acos(c.max())) > 10.0


def test_paper_workload_shapes():
    many, few = synth.cfg_paper(55), synth.cfg_paper(19)
    assert many.geom.n_rays == 55 * 91 * 91 > many.geom.n_voxels == 64 ** 3
    assert few.geom.n_rays == 19 * 91 * 91 < few.geom.n_voxels  # fewer rows than columns
