"""Pins for the oracle's projector A and its transpose (CPU only).

A is the paper's system matrix (Sec. II-A, eq. 1); its discretisation is not
given there, so the reading is the exact path length of one ray per detector
pixel centre through each unit voxel (Siddon).  The oracle's Siddon walk is
pinned against an independent brute-force slab intersection of every
(ray, voxel) pair, against chord lengths computed here from face
intersections, against closed forms for axis-aligned rays, and against the
analytic image position of a single voxel.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def small_geoms():
    par = synth.Geometry(8, 8, 8, np.array([0.3, 1.1, 2.5]), synth.PARALLEL, 12, 8, 1.0, 1.0)
    cone = synth.Geometry(8, 8, 8, np.array([0.2, 2.0, 4.1]), synth.CONE, 12, 12, 1.5, 1.5,
                          32.0, 48.0)
    # non-cubic volumes catch any transposition of the (x, y, z) index order
    par_nc = synth.Geometry(7, 8, 5, np.array([0.0, 0.7, 1.9, math.pi / 2]), synth.PARALLEL,
                            13, 7, 1.0, 1.0)
    cone_nc = synth.Geometry(6, 9, 7, np.array([0.4, 1.7, 3.3, 5.0]), synth.CONE, 16, 11,
                             1.3, 1.2, 30.0, 50.0)
    return {"par": par, "cone": cone, "par_nc": par_nc, "cone_nc": cone_nc}


GEOMS = small_geoms()


@pytest.mark.parametrize("name", list(GEOMS))
def test_siddon_equals_bruteforce_slab(name):
    g = GEOMS[name]
    x = synth.random_volume(g.vol_shape, 11)
    y = oracle.project(g, x)
    yb = oracle.project_bruteforce(g, x)
    assert np.max(np.abs(y - yb)) <= 1e-13 * max(1.0, np.max(np.abs(yb)))
    assert np.count_nonzero(yb) > 0


@pytest.mark.parametrize("name", list(GEOMS))
def test_siddon_matches_dense_matrix_per_entry(name):
    """Each unit vector e_j projects to column j of the slab matrix."""
    g = GEOMS[name]
    A = oracle.matrix_dense(g)
    N = g.n_voxels
    rng = np.random.default_rng(5)
    for j in rng.choice(N, size=min(N, 40), replace=False):
        e = np.zeros(N)
        e[j] = 1.0
        col = oracle.project(g, e.reshape(g.vol_shape)).ravel()
        assert np.max(np.abs(col - A[:, j])) <= 1e-13


def _chord_box(p0, p1, lo, hi):
    """Chord of the infinite line through p0, p1 with the box, from the
    intersection points of the line with the six face rectangles."""
    p0 = np.asarray(p0, float)
    d = np.asarray(p1, float) - p0
    for a in range(3):  # a line inside a face plane: half-open cells
        if d[a] == 0.0 and not (lo[a] <= p0[a] < hi[a]):
            return 0.0
    ts = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        for face in (lo[a], hi[a]):
            t = (face - p0[a]) / d[a]
            q = p0 + t * d
            others = [b for b in range(3) if b != a]
            if all(lo[b] - 1e-12 <= q[b] <= hi[b] + 1e-12 for b in others):
                ts.append(t)
    if len(ts) < 2:
        return 0.0
    return (max(ts) - min(ts)) * float(np.linalg.norm(d))


@pytest.mark.parametrize("name", list(GEOMS))
def test_ray_sum_of_ones_is_chord_length(name):
    g = GEOMS[name]
    ones = np.ones(g.vol_shape)
    y = oracle.project(g, ones)
    lo = [-g.nx / 2, -g.ny / 2, -g.nz / 2]
    hi = [g.nx / 2, g.ny / 2, g.nz / 2]
    for v in range(g.n_views):
        for row in range(g.det_rows):
            for col in range(g.det_cols):
                p0, p1 = oracle.ray_endpoints(g, v, row, col)
                c = _chord_box(p0, p1, lo, hi)
                assert abs(y[v, row, col] - c) <= 1e-11 * max(1.0, c), (v, row, col)


def test_axis_aligned_parallel_rays():
    """theta = 0: rays run along +x through (y, z) = (u, w), so each ray sum
    is the plain sum of one x-row of voxels; theta = pi/2: rays run along y
    at x = -u."""
    n = 8
    g = synth.Geometry(n, n, n, np.array([0.0, math.pi / 2]), synth.PARALLEL, 10, 8, 1.0, 1.0)
    x = synth.random_volume(g.vol_shape, 3)
    y = oracle.project(g, x)
    for row in range(g.det_rows):
        w = row - (g.det_rows - 1) / 2
        k = math.floor(w + n / 2)
        for col in range(g.det_cols):
            u = col - (g.det_cols - 1) / 2
            j = math.floor(u + n / 2)
            exp0 = x[k, j, :].sum() if 0 <= j < n and 0 <= k < n else 0.0
            assert abs(y[0, row, col] - exp0) <= 1e-12
            i = math.floor(-u + n / 2)
            exp1 = x[k, :, i].sum() if 0 <= i < n and 0 <= k < n else 0.0
            assert abs(y[1, row, col] - exp1) <= 1e-12


@pytest.mark.parametrize("cone", [False, True])
def test_single_voxel_images_where_predicted(cone):
    """A single voxel's projection is centred on the analytic image of its
    centre: u = p.e_u (parallel) or SDD (p.e_u) / (R - p.e_s) (cone)."""
    n = 16
    ang = np.array([0.0, 0.9, 2.2, 4.0])
    if cone:
        g = synth.cone_geometry(n, 4, 24, 24, 1.5, 4 * n, 6 * n, angles=ang)
    else:
        g = synth.parallel_geometry(n, 4, 24, 16, angles=ang)
    for (i, j, k) in [(11, 3, 5), (2, 13, 12), (8, 8, 2)]:
        x = np.zeros(g.vol_shape)
        x[k, j, i] = 1.0
        y = oracle.project(g, x)
        p = np.array([i + 0.5 - n / 2, j + 0.5 - n / 2, k + 0.5 - n / 2])
        for v, th in enumerate(ang):
            es = np.array([math.cos(th), math.sin(th), 0.0])
            eu = np.array([-math.sin(th), math.cos(th), 0.0])
            a, b = p @ eu, p @ es
            if cone:
                mag = g.src_to_det / (g.src_to_centre - b)
                u, w = a * mag, p[2] * mag
            else:
                u, w = a, p[2]
            colc = u / g.pitch_u + (g.det_cols - 1) / 2
            rowc = w / g.pitch_v + (g.det_rows - 1) / 2
            img = y[v]
            tot = img.sum()
            assert tot > 0
            rr, cc = np.mgrid[0:img.shape[0], 0:img.shape[1]]
            cr, ccol = (rr * img).sum() / tot, (cc * img).sum() / tot
            assert abs(ccol - colc) < 0.5 and abs(cr - rowc) < 0.5, (v, ccol, colc, cr, rowc)
            assert img[int(round(rowc)), int(round(colc))] > 0


@pytest.mark.parametrize("name", list(GEOMS))
def test_backprojection_is_transpose_of_dense_matrix(name):
    g = GEOMS[name]
    A = oracle.matrix_dense(g)
    r = np.random.default_rng(8).standard_normal(g.proj_shape)
    xb = oracle.backproject(g, r).ravel()
    ref = A.T @ r.ravel()
    assert np.max(np.abs(xb - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("wl", ["small_parallel", "cone64"])
def test_adjoint_identity_workloads(wl):
    w = synth.cfg_small_parallel() if wl == "small_parallel" else synth.cfg_cone64()
    g = w.geom
    rng = np.random.default_rng(21)
    x = rng.standard_normal(g.vol_shape)
    r = rng.standard_normal(g.proj_shape)
    lhs = float(np.sum(oracle.project(g, x) * r))
    rhs = float(np.sum(x * oracle.backproject(g, r)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 10
    assert abs(lhs - rhs) / (np.linalg.norm(x) * np.linalg.norm(r)) <= 1e-12


def test_half_open_cells_for_rays_in_voxel_faces():
    """A parallel ray lying exactly in the plane z = 0 (odd detector row
    count puts a row centre there, even nz puts a voxel face there) belongs
    to the voxel layer above the face, k = nz/2."""
    n = 6
    g = synth.Geometry(n, n, n, np.array([0.4]), synth.PARALLEL, 9, 7, 1.0, 1.0)
    x = np.zeros(g.vol_shape)
    x[n // 2] = 1.0  # layer k = 3 spans z in [0, 1)
    y = oracle.project(g, x)
    ones = oracle.project(g, np.ones(g.vol_shape))
    mid = (g.det_rows - 1) // 2
    assert np.allclose(y[0, mid], ones[0, mid])
    x2 = np.zeros(g.vol_shape)
    x2[n // 2 - 1] = 1.0  # layer below the face sees nothing from that row
    assert np.all(oracle.project(g, x2)[0, mid] == 0.0)


def test_nnz_counts_positive_lengths():
    g = GEOMS["cone"]
    A = oracle.matrix_dense(g)
    assert oracle.nnz(g) == int(np.count_nonzero(A > 0))
