"""Pins for the oracle's smoothed total variation (CPU only).

Eq. 2 defines TV as the sum over voxels of the Euclidean norm of the
forward-difference gradient D_j x.  The methods need a Lipschitz gradient, so
the norm is Huber-smoothed with parameter tau; differences that would reach
outside the volume are zero (reflecting boundary).  Pins: the closed-form TV
of an axis-aligned box (derived in the docstring), central finite
differences, translation invariance, a zero-sum gradient, the quadratic
regime equal to the graph Laplacian / tau, and the gradient-map closed form
of eq. 10.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def box_tv_interior(a, b, d, c, tau):
    """Box of a x b x d voxels (x, y, z extents) of value c >= tau, strictly
    inside a zero volume.  Nonzero D_j x occur at
      - the voxel just below each lower face: one component c -> ab+bd+ad voxels;
      - box voxels on the upper faces: a voxel on s upper faces has s
        components -c, norm c*sqrt(s):  s=1: (b-1)(d-1)+(a-1)(d-1)+(a-1)(b-1),
        s=2: (a-1)+(b-1)+(d-1), s=3: 1.
    Every nonzero norm is >= c >= tau, so each such voxel gives |z| - tau/2
    and every zero voxel gives 0."""
    n1 = a * b + b * d + a * d + (b - 1) * (d - 1) + (a - 1) * (d - 1) + (a - 1) * (b - 1)
    n2 = (a - 1) + (b - 1) + (d - 1)
    n3 = 1
    tv = c * (n1 + math.sqrt(2) * n2 + math.sqrt(3) * n3)
    return tv, tv - 0.5 * tau * (n1 + n2 + n3)


@pytest.mark.parametrize("a,b,d", [(1, 1, 1), (3, 2, 4), (5, 5, 2)])
def test_box_closed_form_interior(a, b, d):
    tau, c = 1e-4, 0.7
    x = np.zeros((9, 8, 10))
    x[2:2 + d, 1:1 + b, 3:3 + a] = c
    tv0, tvt = box_tv_interior(a, b, d, c, tau)
    T = oracle.tv(x, tau, grad=False)
    assert abs(T - tvt) <= 1e-12 * tvt
    T0 = oracle.tv(x, 1e-300, grad=False)
    assert abs(T0 - tv0) <= 1e-12 * tv0


def test_box_touching_upper_x_face_reflecting_boundary():
    """Box occupying the last a x-layers: its voxels on the upper x face have
    no x difference (neighbour outside the volume).  Nonzero norms: lower
    faces ab+bd+ad (one component each); box voxels on the upper y face
    only a(d-1), upper z only a(b-1) (norm c); on both a (norm c sqrt 2)."""
    a, b, d, c, tau = 3, 4, 2, 0.5, 1e-4
    nx = 7
    x = np.zeros((6, 8, nx))
    x[1:1 + d, 2:2 + b, nx - a:] = c
    n1 = a * b + b * d + a * d + a * (d - 1) + a * (b - 1)
    n2 = a
    tv = c * (n1 + math.sqrt(2) * n2)
    T = oracle.tv(x, tau, grad=False)
    assert abs(T - (tv - 0.5 * tau * (n1 + n2))) <= 1e-12 * tv


def _volume_away_from_tau(shape, seed, tau):
    rng = np.random.default_rng(seed)
    while True:
        x = rng.uniform(0, 1, size=shape)
        nz, ny, nx = shape
        dx = np.zeros(shape)
        dy = np.zeros(shape)
        dz = np.zeros(shape)
        dx[:, :, :-1] = np.diff(x, axis=2)
        dy[:, :-1, :] = np.diff(x, axis=1)
        dz[:-1, :, :] = np.diff(x, axis=0)
        nrm = np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
        # keep every |D_j x| far from the kink (the corner voxel has 0 < tau)
        inner = nrm.ravel()[:-1]
        if np.min(inner) > 100 * tau:
            return x


@pytest.mark.parametrize("shape", [(4, 4, 4), (5, 6, 4), (6, 5, 6)])
def test_tv_gradient_central_differences(shape):
    tau = 1e-4
    x = _volume_away_from_tau(shape, 7, tau)
    T, g = oracle.tv(x, tau)
    h = 1e-6
    fd = np.zeros_like(x)
    for j in range(x.size):
        e = np.zeros(x.size)
        e[j] = h
        e = e.reshape(shape)
        fd.ravel()[j] = (oracle.tv(x + e, tau, grad=False) - oracle.tv(x - e, tau, grad=False)) / (2 * h)
    err = np.max(np.abs(fd - g)) / np.max(np.abs(g))
    assert err <= 1e-7


def test_tv_translation_invariance_and_zero_sum_gradient():
    tau = 1e-3
    x = synth.random_volume((6, 7, 5), 2)
    T, g = oracle.tv(x, tau)
    T2, g2 = oracle.tv(x + 3.25, tau)
    assert abs(T - T2) <= 1e-12 * T
    assert np.max(np.abs(g - g2)) <= 1e-12
    assert abs(g.sum()) <= 1e-11 * np.abs(g).sum()


def _neumann_laplacian(x):
    """Graph Laplacian of the 6-neighbour grid: sum over in-volume neighbours
    k of (x_j - x_k)."""
    out = np.zeros_like(x)
    for ax in range(3):
        d = np.diff(x, axis=ax)  # x_{j+1} - x_j on each edge
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        out[tuple(sl_lo)] -= d
        out[tuple(sl_hi)] += d
    return out


def test_quadratic_regime_is_laplacian_over_tau():
    tau = 1.0
    x = 0.01 * synth.random_volume((5, 4, 6), 4)  # every |D_j x| < tau
    T, g = oracle.tv(x, tau)
    ref = _neumann_laplacian(x) / tau
    assert np.max(np.abs(g - ref)) <= 1e-14
    # T = |Dx|^2 / (2 tau) = x^T L x / (2 tau)
    assert abs(T - float(np.sum(x * _neumann_laplacian(x))) / (2 * tau)) <= 1e-14


def test_huber_matches_plain_tv_far_from_kink():
    tau = 1e-8
    x = _volume_away_from_tau((4, 5, 4), 9, tau)
    T = oracle.tv(x, tau, grad=False)
    T0 = oracle.tv(x, 1e-300, grad=False)
    # corner voxel (all differences outside) contributes 0 to both
    assert abs(T0 - T - 0.5 * tau * (x.size - 1)) <= 1e-12 * T0


def test_gradient_map_closed_form():
    """For x >= 0: G_nu(x)_i = nu (x_i - max(x_i - g_i / nu, 0)) = min(g_i, nu x_i)."""
    rng = np.random.default_rng(3)
    x = np.maximum(rng.standard_normal(500), 0.0)
    g = rng.standard_normal(500)
    for nu in (0.3, 1.0, 17.0):
        ref = np.linalg.norm(np.minimum(g, nu * x))
        assert abs(oracle.gradmap_norm(x, g, nu) - ref) <= 1e-13 * ref


def test_gradient_map_zero_iff_kkt():
    x = np.array([0.0, 0.0, 2.0, 5.0])
    g = np.array([1.0, 0.5, 0.0, 0.0])   # x >= 0, g >= 0, x*g = 0
    assert oracle.gradmap_norm(x, g, 2.0) == 0.0
    g2 = g.copy()
    g2[2] = 1e-3                          # complementarity broken
    assert oracle.gradmap_norm(x, g2, 2.0) > 0.0


def _huber(z, tau):
    n = np.linalg.norm(z)
    return n - tau / 2 if n >= tau else n * n / (2 * tau)


def _huber_grad(z, tau):
    return z / max(tau, np.linalg.norm(z))


@pytest.mark.parametrize("regime", ["quad", "lin", "a_lin_b_quad", "a_quad_b_lin"])
def test_huber_bregman_matches_definition(regime):
    """Per-regime cancellation-free Bregman distance of Phi_tau equals
    Phi(a) - Phi(b) - grad Phi(b)^T (a - b) and is nonnegative."""
    tau = 0.1
    rng = np.random.default_rng(hash(regime) % 2**32)
    scale = {"quad": (0.3, 0.3), "lin": (3.0, 3.0), "a_lin_b_quad": (3.0, 0.3),
             "a_quad_b_lin": (0.3, 3.0)}[regime]
    for _ in range(200):
        a = rng.standard_normal(3)
        b = rng.standard_normal(3)
        a *= scale[0] * tau / np.linalg.norm(a) * rng.uniform(0.2, 0.99 if scale[0] < 1 else 3)
        b *= scale[1] * tau / np.linalg.norm(b) * rng.uniform(0.2, 0.99 if scale[1] < 1 else 3)
        ref = _huber(a, tau) - _huber(b, tau) - _huber_grad(b, tau) @ (a - b)
        val = oracle.huber_bregman(a, b, a - b, tau)
        assert val >= 0.0
        assert abs(val - ref) <= 1e-12 * max(1.0, abs(_huber(a, tau)))


def test_tv_bregman_sums_voxel_terms():
    tau = 1e-2
    x = synth.random_volume((5, 6, 4), 21)
    y = synth.random_volume((5, 6, 4), 22)
    Tx = oracle.tv(x, tau, grad=False)
    Ty, gy = oracle.tv(y, tau)
    ref = Tx - Ty - float(np.sum(gy * (x - y)))
    assert abs(oracle.tv_bregman(x, y, tau) - ref) <= 1e-11 * Tx


def test_tv_bregman_small_perturbation_is_accurate():
    """For x = y + h v the Bregman distance is O(h^2); the per-voxel form
    resolves it where T(x) - T(y) - grad^T (x - y) is pure rounding."""
    tau = 1e-4
    y = _volume_away_from_tau((5, 5, 5), 3, tau)
    v = synth.random_volume((5, 5, 5), 4, -1, 1)
    b1 = oracle.tv_bregman(y + 1e-6 * v, y, tau)
    b2 = oracle.tv_bregman(y + 2e-6 * v, y, tau)
    assert b1 > 0
    assert abs(b2 / b1 - 4.0) <= 1e-6
