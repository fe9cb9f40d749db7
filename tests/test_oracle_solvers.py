"""Pins for the oracle's GP, GPBB and UPN solvers (CPU only).

GP is eq. 6 with the step 1/L_k from BT (Alg. 2); GPBB is Alg. 1; UPN is
Alg. 3 with the mu estimate of eq. 9; all stop on the gradient map of
eq. 10 (Sec. III-D).  Pins: with alpha = 0 the problem is nonnegative least
squares, solved independently by scipy's Lawson-Hanson NNLS; all three
methods must reach the same minimiser; the L / mu / theta invariants;
UPN with mu_k forced to L_k is GP step for step; UPN with mu = 0 follows the
textbook accelerated-gradient (FISTA) momentum recurrence.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_overdetermined_geom():
    # 4^3 voxels, 6 cone views of 8 x 8 pixels: 384 rays > 64 unknowns
    return synth.cone_geometry(4, 6, 8, 8, 1.5, 16.0, 24.0)


def _nnls_bound(A, eps, gm0):
    """With alpha = 0 the objective is strongly convex with modulus
    lambda_min(A^T A); a point whose gradient map is below eps * gm0 lies
    within 2 eps gm0 / lambda_min of the minimiser."""
    lam_min = np.linalg.svd(A, compute_uv=False).min() ** 2
    return 2.0 * eps * gm0 / lam_min


@pytest.mark.parametrize("method", [oracle.GP, oracle.GPBB, oracle.UPN])
def test_alpha_zero_matches_scipy_nnls_geometry(method):
    """eps = 1e-8: below about 1e-9 the literal BT test of Alg. 2 compares
    objective values that agree to the last FP64 digits, so the oracle (which
    keeps the printed form) is only asked for what FP64 can resolve."""
    g = tiny_overdetermined_geom()
    A = oracle.matrix_dense(g)
    assert np.linalg.matrix_rank(A) == A.shape[1]
    x_true = synth.random_volume(g.vol_shape, 12, -0.5, 1.0)  # some negative -> active bounds
    b = A @ x_true.ravel() + 0.05 * np.random.default_rng(13).standard_normal(A.shape[0])
    x_ref, _ = nnls(A, b, maxiter=5000)
    eps = 1e-8
    x, info, _ = oracle.solve(g, b.reshape(g.proj_shape), method=method, alpha=0.0,
                              eps=eps, max_iter=200000)
    assert info["status"] == oracle.CONVERGED
    bound = _nnls_bound(A, eps, info["gm0"])
    assert np.linalg.norm(x.ravel() - x_ref) <= bound
    assert bound < 2e-4
    assert np.any(x_ref == 0.0)


@pytest.mark.parametrize("method", [oracle.GP, oracle.GPBB, oracle.UPN])
def test_alpha_zero_matches_scipy_nnls_dense(method):
    rng = np.random.default_rng(31)
    A = rng.standard_normal((60, 27))
    b = rng.standard_normal(60)
    x_ref, _ = nnls(A, b)
    eps = 1e-7
    x, info, _ = oracle.solve_dense(A, b, (3, 3, 3), method=method, alpha=0.0, eps=eps,
                                    max_iter=200000)
    assert info["status"] == oracle.CONVERGED
    # BT stayed within rho_L of the true Lipschitz constant (no FP64 breakdown)
    assert info["L"] <= 2.0 * np.linalg.svd(A, compute_uv=False).max() ** 2 * (1 + 1e-12)
    bound = _nnls_bound(A, eps, info["gm0"])
    assert np.linalg.norm(x.ravel() - x_ref) <= bound
    assert bound < 1e-5
    assert np.any(x_ref == 0.0)


@pytest.fixture(scope="module")
def small_problem():
    w = synth.cfg_small_parallel()
    g = oracle.Geometry(w.geom)
    x_true = w.phantom()
    b = oracle.noisy_data(g, x_true, w.unit_noise(), w.eta)
    return w, g, b, x_true


@pytest.fixture(scope="module")
def small_reference(small_problem):
    """phi* and x* from UPN at a tolerance 100x below the one compared
    (the paper's own technique, Sec. IV-B)."""
    w, g, b, _ = small_problem
    x, info, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-10,
                              max_iter=20000)
    assert info["status"] == oracle.CONVERGED
    return x, info


@pytest.mark.parametrize("method", [oracle.GPBB, oracle.UPN])
def test_methods_reach_same_minimiser(small_problem, small_reference, method):
    w, g, b, _ = small_problem
    x_star, info_star = small_reference
    x, info, _ = oracle.solve(g, b, method=method, alpha=w.alpha, tau=w.tau, eps=1e-8,
                              max_iter=20000)
    assert info["status"] == oracle.CONVERGED
    rel = np.linalg.norm(x - x_star) / np.linalg.norm(x_star)
    assert rel <= 1e-4
    assert abs(info["phi"] - info_star["phi"]) <= 1e-8 * info_star["phi"]
    assert np.all(x >= 0)


def test_gp_converges_towards_same_minimiser(small_problem, small_reference):
    """GP is slow (the paper's point); after a fixed budget it must be
    monotone and approaching phi*."""
    w, g, b, _ = small_problem
    x_star, info_star = small_reference
    x, info, h = oracle.solve(g, b, method=oracle.GP, alpha=w.alpha, tau=w.tau, eps=1e-8,
                              max_iter=3000, hist_len=3000)
    phi = h["phi"][:info["iters"]]
    assert np.all(np.diff(phi) <= 1e-12 * phi[0])      # BT-GP is a descent method
    assert info["status"] == oracle.NOTCONV             # GP is far slower (Sec. IV-B)
    gap = (phi - info_star["phi"]) / info_star["phi"]
    assert gap[-1] <= 0.05 and gap[-1] < 1e-3 * gap[0]
    assert info["phi"] >= info_star["phi"] * (1 - 1e-12)


def test_upn_invariants(small_problem):
    w, g, b, _ = small_problem
    x, info, h = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-6,
                              max_iter=5000, hist_len=5000)
    n = info["iters"]
    L = h["L"][:n]
    mu = h["mu"][:n - 1]   # the stopping iteration ends before its mu update
    assert np.all(np.diff(L) >= 0)                    # BT never lowers L (Alg. 2/3)
    assert np.all(mu >= 0) and np.all(np.diff(mu) <= 0)  # eq. 9 makes mu non-increasing
    assert mu[0] == pytest.approx(L[0] / 4)
    # L bounded by rho_L times the gradient's Lipschitz constant:
    # |A|^2 (power iteration) + alpha * 12 / tau  (|D|^2 <= 12)
    A_lam = _power_iteration(g)
    assert L[-1] <= 2.0 * (A_lam + w.alpha * 12.0 / w.tau) * (1 + 1e-9)
    gm = h["gm"][:n]
    assert gm[-1] <= 1e-6


def _power_iteration(g, iters=60):
    x = np.random.default_rng(1).standard_normal(g.vol_shape)
    lam = 0.0
    for _ in range(iters):
        y = oracle.backproject(g, oracle.project(g, x))
        lam = np.linalg.norm(y) / np.linalg.norm(x)
        x = y / np.linalg.norm(y)
    return lam


def test_upn_with_mu_equal_L_is_gp(small_problem):
    """mu_k := L_k gives theta = 1 and beta = 0 in Alg. 3, so y = x and every
    UPN step is a GP step with the same BT."""
    w, g, b, _ = small_problem
    x1, i1, h1 = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-4,
                              max_iter=300, force_mu=1, hist_len=300)
    x2, i2, h2 = oracle.solve(g, b, method=oracle.GP, alpha=w.alpha, tau=w.tau, eps=1e-4,
                              max_iter=300, hist_len=300)
    assert np.array_equal(x1, x2)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(h1["phi"], h2["phi"])


def test_upn_with_mu_zero_is_fista(small_problem):
    """mu = 0: theta_{k+1}^2 = (1 - theta_{k+1}) theta_k^2 and
    beta_k = theta_k (1 - theta_k) / (theta_k^2 + theta_{k+1}), which equals
    the FISTA momentum (t_k - 1) / t_{k+1}, t = 1/theta,
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 (Beck & Teboulle 2009).  The
    iteration below is that textbook method with the same backtracking,
    built on the oracle's phi and gradient only."""
    w, g, b, _ = small_problem
    K = 25
    xo, io, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-30,
                             max_iter=K, force_mu=2)
    f = lambda z: oracle.phi(g, b, w.alpha, w.tau, z)
    fg = lambda z: oracle.phi_grad(g, b, w.alpha, w.tau, z)

    def bt(y, Lbar):
        fy, gy = fg(y)
        L = Lbar
        while True:
            x = np.maximum(y - gy / L, 0.0)
            if f(x) <= fy + np.sum(gy * (x - y)) + 0.5 * L * np.sum((x - y) ** 2):
                return x, L
            L *= 2.0

    x0 = np.zeros(g.vol_shape)
    x, L = bt(x0, 1.0)
    y = x.copy()
    t = 1.0  # theta_1 = sqrt(mu_0 / L_0) = 1 with mu_0 = L_0
    xprev = x
    for k in range(1, K):
        xn, L = bt(y, L)
        tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
        beta = (t - 1) / tn
        t = tn
        y = xn + beta * (xn - xprev)
        xprev = xn
    assert np.max(np.abs(xprev - xo)) <= 1e-9 * np.max(np.abs(xo))


def test_paper_parameter_defaults():
    """Parameter values the paper prints (golden file with citations)."""
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as fh:
        gold = json.load(fh)
    p = oracle.default_params(oracle.GPBB, alpha=gold["alpha"]["value"])
    assert p["gpbb_K"] == gold["gpbb_K"]["value"]
    assert p["gpbb_sigma"] == gold["gpbb_sigma"]["value"]
    assert p["gpbb_beta0"] == gold["gpbb_beta0"]["value"]
    assert gold["gpbb_theta0"]["value"] == 1.0


def test_stop_mode_absolute(small_problem):
    """Sec. III-D as printed: stop when |G_nu(x)|_2 / N <= eps."""
    w, g, b, _ = small_problem
    N = w.geom.n_voxels
    x, info, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-6,
                              stop_mode=1, max_iter=20000)
    assert info["status"] == oracle.CONVERGED
    assert info["gm"] / N <= 1e-6


def test_bt_cap_reports_stall(small_problem):
    w, g, b, _ = small_problem
    x, info, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-6,
                              max_trials=2, L_bar=1e-6, max_iter=100)
    assert info["status"] == oracle.STALL
    assert np.all(x == 0.0)   # nothing accepted: the start point is returned


def test_bregman_form_bt_takes_same_steps(small_problem):
    """bt_form = 1 evaluates the same BT inequality (Alg. 2) and the same
    eq. 9 numerator, so the two forms take the same decisions until a near
    tie is rounded differently (here after ~150 iterations); both then go on
    to the same minimiser."""
    w, g, b, _ = small_problem
    K = 120
    x0, i0, h0 = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-30,
                              max_iter=K, hist_len=K)
    x1, i1, h1 = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-30,
                              max_iter=K, hist_len=K, bt_form=1)
    assert i0["iters"] == i1["iters"] == K
    assert i0["func_evals"] == i1["func_evals"]
    assert np.array_equal(h0["L"], h1["L"])
    # the printed eq. 9 numerator f(x) - f(y) - grad^T (x - y) loses ~5 digits
    # to cancellation here; the Bregman form does not
    rel_mu = np.abs(h0["mu"][:K - 1] - h1["mu"][:K - 1]) / h1["mu"][:K - 1]
    assert np.max(rel_mu) <= 1e-4
    # ... and the momentum amplifies that mu difference in the iterates
    assert np.max(np.abs(x0 - x1)) <= 1e-3 * np.max(np.abs(x1))
    xa, ia, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-8,
                             max_iter=20000)
    xb, ib, _ = oracle.solve(g, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-8,
                             max_iter=20000, bt_form=1)
    assert ia["status"] == ib["status"] == oracle.CONVERGED
    assert np.linalg.norm(xa - xb) <= 1e-4 * np.linalg.norm(xa)


@pytest.mark.parametrize("method", [oracle.GP, oracle.UPN])
def test_bregman_form_reaches_tight_nnls_tolerance(method):
    """Where the printed test breaks down in FP64 (eps = 1e-11, see the
    dense NNLS pin), the Bregman form still resolves the BT decision."""
    rng = np.random.default_rng(31)
    A = rng.standard_normal((60, 27))
    b = rng.standard_normal(60)
    x_ref, _ = nnls(A, b)
    eps = 1e-11
    x, info, _ = oracle.solve_dense(A, b, (3, 3, 3), method=method, alpha=0.0, eps=eps,
                                    max_iter=200000, bt_form=1)
    assert info["status"] == oracle.CONVERGED
    assert info["L"] <= 2.0 * np.linalg.svd(A, compute_uv=False).max() ** 2 * (1 + 1e-12)
    assert np.linalg.norm(x.ravel() - x_ref) <= _nnls_bound(A, eps, info["gm0"])
