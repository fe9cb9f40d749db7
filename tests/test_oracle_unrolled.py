"""Pins of the oracle's differentiated form (TV Hessian-vector product and the
reverse-mode gradient of K unrolled UPN steps), none of which re-derives the
oracle's own code:

* H(y) v against central differences of the TV gradient, its symmetry, and
  the quadratic regime where it is the Neumann Laplacian over tau;
* the unrolled forward map against the UPN solver run for K iterations
  (same steps, bit for bit);
* K = 1, where x^(1) = P_Q(A^T b / L_0) and the gradient has a closed form;
* central differences of the replayed forward map (L decisions held fixed)
  on smooth pieces: the step is kept small enough that every projection
  mask and Huber regime is the same at both ends (checked through the
  forward pass's pattern signature), so the difference quotient converges
  to the derivative and a dropped term or wrong sign shows as an O(1) error.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def neumann_laplacian(v):
    """D^T D v with forward differences, zero across the upper faces."""
    out = np.zeros_like(v)
    for ax in range(3):
        d = np.diff(v, axis=ax)  # D v along ax (upper-face difference dropped)
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        out[tuple(sl_lo)] -= d
        out[tuple(sl_hi)] += d
    return out


@pytest.mark.parametrize("tau", [1e-4, 0.3, 10.0])
def test_tv_hessvec_matches_central_differences(tau):
    rng = np.random.default_rng(11)
    y = rng.uniform(0.0, 1.0, (5, 6, 7))
    v = rng.standard_normal(y.shape)
    H = oracle.tv_hessvec(y, v, tau)
    h = 1e-6
    fd = (oracle.tv(y + h * v, tau)[1] - oracle.tv(y - h * v, tau)[1]) / (2 * h)
    assert np.linalg.norm(H - fd) <= 1e-7 * np.linalg.norm(fd)


def test_tv_hessvec_symmetric():
    rng = np.random.default_rng(12)
    y = rng.uniform(0.0, 1.0, (4, 5, 6))
    u = rng.standard_normal(y.shape)
    v = rng.standard_normal(y.shape)
    for tau in (1e-4, 0.2):
        a = np.sum(oracle.tv_hessvec(y, u, tau) * v)
        b = np.sum(u * oracle.tv_hessvec(y, v, tau))
        assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


def test_tv_hessvec_quadratic_regime_is_laplacian():
    rng = np.random.default_rng(13)
    y = 1e-3 * rng.uniform(0.0, 1.0, (4, 6, 5))  # all |D_j y| < tau
    v = rng.standard_normal(y.shape)
    tau = 0.5
    H = oracle.tv_hessvec(y, v, tau)
    np.testing.assert_allclose(H, neumann_laplacian(v) / tau, rtol=0, atol=1e-12)


@pytest.fixture(scope="module")
def small_cone():
    n = 10
    geom = synth.cone_geometry(n, 6, 16, 16, 1.5, 4 * n, 6 * n)
    og = oracle.Geometry(geom)
    xt = synth.ellipsoid_phantom(n, 4, 7)
    b = oracle.noisy_data(og, xt, synth.unit_noise(og.proj_shape, 8), 0.01)
    return og, xt, b


@pytest.mark.parametrize("K", [1, 2, 7])
def test_unrolled_forward_equals_upn_solver(small_cone, K):
    og, xt, b = small_cone
    r = oracle.unrolled(og, b, K, 1e-2)
    x, info, hist = oracle.solve(og, b, method=oracle.UPN, alpha=1e-2, eps=0.0, max_iter=K,
                                 bt_form=1, hist_len=K)
    assert r["status"] == 0 and info["iters"] == K
    assert np.array_equal(r["xK"], x)
    np.testing.assert_array_equal(r["L"], hist["L"][:K])
    # replaying the recorded L reproduces the same map
    r2 = oracle.unrolled(og, b, K, 1e-2, L=r["L"])
    assert np.array_equal(r2["xK"], r["xK"])


def test_unrolled_k1_closed_form(small_cone):
    og, xt, b = small_cone
    r = oracle.unrolled(og, b, 1, 1e-2)
    L0 = r["L"][0]
    x1 = np.maximum(oracle.backproject(og, b) / L0, 0.0)  # grad T(0) = 0
    np.testing.assert_allclose(r["xK"], x1, rtol=1e-13, atol=1e-15)
    xb = 2.0 * (x1 - xt)
    g = oracle.unrolled(og, b, 1, 1e-2, L=r["L"], xK_bar=xb)
    expect_b = oracle.project(og, np.where(x1 > 0, xb, 0.0)) / L0
    np.testing.assert_allclose(g["b_bar"], expect_b, rtol=1e-12, atol=1e-14)
    assert g["alpha_bar"] == 0.0


def fd_check(og, xt, b, K, alpha, tau, h):
    base = oracle.unrolled(og, b, K, alpha, tau=tau)
    assert base["status"] == 0
    L = base["L"]
    g = oracle.unrolled(og, b, K, alpha, tau=tau, L=L, xK_bar=2.0 * (base["xK"] - xt))
    w = synth.fd_direction(og.proj_shape, 503)
    rms = math.sqrt(float(np.mean(b * b)))

    def run(a, bb):
        r = oracle.unrolled(og, bb, K, a, tau=tau, L=L)
        return float(np.sum((r["xK"] - xt) ** 2)), r["signature"]

    lp, sp = run(alpha * math.exp(h), b)
    lm, sm = run(alpha * math.exp(-h), b)
    fd_a = (lp - lm) / (2 * h)
    e = h * rms
    lp, sp2 = run(alpha, b + e * w)
    lm, sm2 = run(alpha, b - e * w)
    fd_b = (lp - lm) / (2 * e)
    same = sp == sm == sp2 == sm2 == base["signature"]
    return dict(adj_a=alpha * g["alpha_bar"], fd_a=fd_a, adj_b=float(np.sum(g["b_bar"] * w)),
                fd_b=fd_b, same=same, states=base["mu_state"])


@pytest.mark.parametrize("K,alpha,tau", [(30, 1e-2, 1e-2), (10, 1e-2, 1e-4)])
def test_unrolled_adjoint_matches_central_differences(small_cone, K, alpha, tau):
    og, xt, b = small_cone
    r = fd_check(og, xt, b, K, alpha, tau, 1e-6)
    assert r["same"], "difference interval crosses a mask or regime change"
    assert (r["states"] == 1).sum() >= 3  # the eq. 9 branch is differentiated too
    assert abs(r["adj_a"] - r["fd_a"]) <= 1e-6 * abs(r["adj_a"])
    assert abs(r["adj_b"] - r["fd_b"]) <= 1e-6 * abs(r["adj_b"])


@pytest.mark.parametrize("alpha,h", [(1e-2, 1e-8), (1e-3, 1e-7)])
def test_unrolled_adjoint_k30_across_regime_changes(small_cone, alpha, h):
    """K = 30, tau = 1e-4: the map is still locally linear but a difference
    interval meets a few Huber-regime or mask switches, each adding O(h)
    error to the quotient, while rounding adds O(eps |l| / h); the agreement
    is ~1e-6 to 1e-5."""
    og, xt, b = small_cone
    r = fd_check(og, xt, b, 30, alpha, 1e-4, h)
    assert abs(r["adj_a"] - r["fd_a"]) <= 1e-4 * abs(r["adj_a"])
    assert abs(r["adj_b"] - r["fd_b"]) <= 1e-4 * abs(r["adj_b"])
