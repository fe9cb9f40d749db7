"""Seeded synthetic inputs for the TV-regularised CT reconstruction workloads.

This module only *describes* and *draws* inputs: scan geometries, piecewise
constant ellipsoid phantoms, unit-variance noise draws and the solver
parameters of each workload.  It holds none of the reconstruction method's
arithmetic (no projection, no TV, no solver step).  Both the FP64 CPU oracle
and the HIP path consume exactly the arrays produced here.

The paper's own test image (the FORBILD head phantom, Sec. IV-A) is not
available, so seeded axis-aligned ellipsoid phantoms stand in for it.  The
paper's noise model (Sec. IV-A, eq. 11) is b = A x_true + e with
||e|| / ||A x_true|| = eta; here e_i ~ N(0, sigma^2) with
sigma = eta * ||A x_true|| / sqrt(m), so this module supplies the N(0, 1)
draws and the caller scales them once A x_true is known.

Conventions (shared definitions of the *inputs*, stated once here):

* volume x has shape (nz, ny, nx), x fastest; voxel (i, j, k) spans
  [i - nx/2, i + 1 - nx/2] x [j - ny/2, ...] x [k - nz/2, ...] (unit voxels,
  volume centred at the origin);
* projection data has shape (n_views, det_rows, det_cols), column fastest;
* view angles are theta_v = span * v / n_views (span = pi for parallel beam,
  2 pi for cone beam), given explicitly as a float64 array;
* the 3D parallel beam (PARALLEL3D) takes one direction d per view; its
  detector plane passes through the origin with axes e_u = (e_z x d) /
  |e_z x d| (e_x when d is along z) and e_v = d x e_u (for d = (cos, sin, 0)
  these are the parallel beam's axes); its ``angles`` are only a view count.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PARALLEL = 0
CONE = 1
PARALLEL3D = 2  # parallel rays along per-view direction vectors (``dirs``)


@dataclasses.dataclass
class Geometry:
    """Scan geometry description (no derived quantities)."""

    nx: int
    ny: int
    nz: int
    angles: np.ndarray  # float64, radians
    beam: int  # PARALLEL or CONE
    det_cols: int
    det_rows: int
    pitch_u: float = 1.0
    pitch_v: float = 1.0
    src_to_centre: float = 0.0  # cone only
    src_to_det: float = 0.0  # cone only
    dirs: Optional[np.ndarray] = None  # PARALLEL3D only: (n_views, 3) float64 directions

    @property
    def n_views(self) -> int:
        return int(len(self.angles))

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_rays(self) -> int:
        return self.n_views * self.det_rows * self.det_cols

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def proj_shape(self):
        return (self.n_views, self.det_rows, self.det_cols)


@dataclasses.dataclass
class Workload:
    name: str
    geom: Geometry
    n_ellipsoids: int
    eta: float  # relative noise level ||e|| / ||A x_true||
    alpha: float
    tau: float
    phantom_seed: int
    noise_seed: int

    def phantom(self) -> np.ndarray:
        g = self.geom
        assert g.nx == g.ny == g.nz
        return ellipsoid_phantom(g.nx, self.n_ellipsoids, self.phantom_seed)

    def unit_noise(self) -> np.ndarray:
        return unit_noise(self.geom.proj_shape, self.noise_seed)


def view_angles(n_views: int, span: float) -> np.ndarray:
    """theta_v = span * v / n_views for v = 0..n_views-1 (float64)."""
    return np.array([span * v / n_views for v in range(n_views)], dtype=np.float64)


def parallel_geometry(n: int, n_views: int, det_cols: int, det_rows: int,
                      pitch: float = 1.0, span: float = math.pi,
                      angles: Optional[np.ndarray] = None) -> Geometry:
    a = view_angles(n_views, span) if angles is None else np.asarray(angles, np.float64)
    return Geometry(n, n, n, a, PARALLEL, det_cols, det_rows, pitch, pitch)


def cone_geometry(n: int, n_views: int, det_cols: int, det_rows: int,
                  pitch: float, src_to_centre: float, src_to_det: float,
                  span: float = 2 * math.pi,
                  angles: Optional[np.ndarray] = None) -> Geometry:
    a = view_angles(n_views, span) if angles is None else np.asarray(angles, np.float64)
    return Geometry(n, n, n, a, CONE, det_cols, det_rows, pitch, pitch,
                    float(src_to_centre), float(src_to_det))


def sphere_directions(n_views: int) -> np.ndarray:
    """n_views view directions spread evenly over the unit sphere (Sec. IV-A).

    A parallel ray along d and one along -d are the same line, so the
    directions cover the upper hemisphere: the golden-angle spiral with equal
    area per direction, z_k = 1 - (k + 1/2) / n_views and longitude
    k * pi (3 - sqrt 5), k = 0..n_views-1.  Returns (n_views, 3) float64.
    """
    k = np.arange(n_views, dtype=np.float64)
    z = 1.0 - (k + 0.5) / n_views
    lon = k * (math.pi * (3.0 - math.sqrt(5.0)))
    r = np.sqrt(1.0 - z * z)
    return np.ascontiguousarray(np.stack([r * np.cos(lon), r * np.sin(lon), z], axis=1))


def parallel3d_geometry(n: int, dirs: np.ndarray, det_cols: int, det_rows: int,
                        pitch: float = 1.0) -> Geometry:
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    return Geometry(n, n, n, np.zeros(len(d)), PARALLEL3D, det_cols, det_rows, pitch, pitch,
                    dirs=d)


def ellipsoid_phantom(n: int, n_ellipsoids: int, seed: int) -> np.ndarray:
    """Sum of seeded axis-aligned ellipsoids, clipped to [0, 1].

    Per ellipsoid the draws are, in this order, from numpy's PCG64
    ``default_rng(seed)``: centre c ~ U[-0.35n, 0.35n]^3 (x, y, z), semi-axes
    r ~ U[0.08n, 0.30n]^3, intensity v ~ U[0, 1].  A voxel whose centre p has
    sum(((p - c) / r)^2) <= 1 receives +v.  Returns float64 (n, n, n).
    """
    rng = np.random.default_rng(seed)
    ctr = np.arange(n, dtype=np.float64) + 0.5 - n / 2.0
    pz, py, px = np.meshgrid(ctr, ctr, ctr, indexing="ij")
    vol = np.zeros((n, n, n), dtype=np.float64)
    for _ in range(n_ellipsoids):
        c = rng.uniform(-0.35 * n, 0.35 * n, size=3)
        r = rng.uniform(0.08 * n, 0.30 * n, size=3)
        v = rng.uniform(0.0, 1.0)
        inside = (((px - c[0]) / r[0]) ** 2 + ((py - c[1]) / r[1]) ** 2
                  + ((pz - c[2]) / r[2]) ** 2) <= 1.0
        vol[inside] += v
    np.clip(vol, 0.0, 1.0, out=vol)
    return vol


def unit_noise(shape, seed: int) -> np.ndarray:
    """N(0, 1) draws of the given shape from ``default_rng(seed)`` (float64)."""
    return np.random.default_rng(seed).standard_normal(size=shape)


def random_volume(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Uniform test vector (float64) for operator-level tests."""
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# ---------------------------------------------------------------------------
# The five workloads.  Cone beam: source at 4n from the centre, flat detector
# at 6n from the source (magnification 1.5, pixel pitch 1.5 so a pixel maps
# to one voxel at the isocentre).
# ---------------------------------------------------------------------------

def cfg_small_parallel() -> Workload:
    """24^3, parallel beam, 8 views over [0, 180 deg), detector 36 x 24."""
    g = parallel_geometry(24, 8, 36, 24, pitch=1.0, span=math.pi)
    return Workload("parallel24", g, 6, 0.01, 1e-2, 1e-4, 101, 102)


def cfg_cone64(alpha: float = 1e-2) -> Workload:
    """64^3, cone beam, 20 views over [0, 360 deg), detector 96 x 96 @ 1.5."""
    n = 64
    g = cone_geometry(n, 20, 96, 96, 1.5, 4 * n, 6 * n)
    return Workload(f"cone64_a{alpha:g}", g, 10, 0.01, alpha, 1e-4, 201, 202)


def cfg_cone256() -> Workload:
    """256^3, cone beam, 60 views over [0, 360 deg), detector 384 x 256 @ 1.5."""
    n = 256
    g = cone_geometry(n, 60, 384, 256, 1.5, 4 * n, 6 * n)
    return Workload("cone256", g, 24, 0.005, 3e-3, 1e-4, 301, 302)


def cfg_batch(n_problems: int = 32, seed: int = 400) -> List[Workload]:
    """Batch of independent cone-beam problems of uneven size.

    Draws from ``default_rng(seed)``, per problem p in order: cube side
    n ~ U{32, 48, 64, 96, 128}, views V ~ U{10..40}, alpha = 10^U[-4, -1].
    Detector side 1.5 n at pitch 1.5; 8 ellipsoids; seeds 4000+2p / 4001+2p.
    """
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_problems):
        n = int(rng.choice([32, 48, 64, 96, 128]))
        v = int(rng.integers(10, 41))
        alpha = float(10.0 ** rng.uniform(-4.0, -1.0))
        side = (3 * n) // 2
        g = cone_geometry(n, v, side, side, 1.5, 4 * n, 6 * n)
        out.append(Workload(f"batch{p}_n{n}_v{v}", g, 8, 0.01, alpha, 1e-4,
                            4000 + 2 * p, 4001 + 2 * p))
    return out


def cfg_unrolled() -> Workload:
    """64^3, cone beam, 30 views, detector 96 x 96 (differentiated form)."""
    n = 64
    g = cone_geometry(n, 30, 96, 96, 1.5, 4 * n, 6 * n)
    return Workload("unrolled64", g, 10, 0.01, 1e-2, 1e-4, 501, 502)


def cfg_paper(n_views: int = 55) -> Workload:
    """The paper's test problem (Sec. IV-A): a 64^3 volume, a parallel beam
    whose n_views directions are spread over the unit sphere (55: many-view,
    19: few-view), 91 x 91 detector pixels, 1 % noise, alpha = 1e-2.  The
    pitch sqrt(3) 64 / 91 makes the detector cover the volume's circumscribed
    sphere from every direction.  Ten seeded ellipsoids stand in for the
    FORBILD head phantom."""
    n = 64
    g = parallel3d_geometry(n, sphere_directions(n_views), 91, 91, math.sqrt(3.0) * n / 91)
    return Workload(f"paper{n_views}", g, 10, 0.01, 1e-2, 1e-4, 600 + n_views, 700 + n_views)


def fd_direction(shape, seed: int = 503) -> np.ndarray:
    """Unit-RMS random direction used by finite-difference checks."""
    w = np.random.default_rng(seed).standard_normal(size=shape)
    return w / math.sqrt(float(np.mean(w * w)))
