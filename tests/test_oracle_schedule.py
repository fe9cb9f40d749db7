"""Pins for the step rules of the oracle's GPBB (Alg. 1) and UPN (Alg. 3).

Reaching the right minimiser does not pin these rules: any convergent
variant (the other Barzilai-Borwein quotient, a monotone line search, a
different beta update, theta from the previous mu/L) reaches the same point.
So the first test follows GPBB through four steps of a problem small enough
to work out by hand, in exact fractions, and the second checks that every
theta UPN records solves the quadratic of Alg. 3 with the mu_k and L_k of the
same iteration, on a run where both change.
"""
import numpy as np
import pytest

import oracle
import synth


def test_gpbb_four_steps_worked_by_hand():
    r"""GPBB (Alg. 1) with K = 2, sigma = 1/4, beta_0 = 1/2 on

        f(x) = 1/2 |A x - b|^2,  A = diag(1, 3),  b = (-3, 2),  Q = {x >= 0},
        grad f(x) = (x1 + 3, 9 x2 - 6),   x^(0) = (1, 0),  theta_0 = 1.

    (alpha = 0: no TV term.)  beta_0 and sigma are not the paper's 0.95 and
    0.1: halving keeps every number a short fraction.

    k = 0: f(x0) = 8 + 2 = 10, g0 = (4, -6), fhat = 10.
        beta = 1/2: P(x0 - g0/2) = P(-1, 3) = (0, 3), f = 9/2 + 49/2 = 29;
            g0.(x0 - xbar) = 4 + 18 = 22; 29 >= 10 - 22/4: rejected, beta = 1/4.
        beta = 1/4: (0, 3/2), f = 9/2 + 25/8 = 61/8; g0.(x0 - xbar) = 13;
            61/8 >= 10 - 13/4 = 27/4: rejected, beta = (1/4)^2 = 1/16.
        beta = 1/16: (3/4, 3/8), f = 225/32 + 49/128 = 949/128;
            g0.(x0 - xbar) = 13/4; 949/128 < 10 - 13/16: accepted.
        (With beta <- beta * beta_0 instead of beta^2 the third trial is
        (1/2, 3/4), f = 1227/128.)
    k = 1: x1 = (3/4, 3/8), g1 = (15/4, -21/8); s = x1 - x0 = (-1/4, 3/8),
        dg = g1 - g0 = (-1/4, 27/8); |s|^2 = 13/64, <s, dg> = 85/64:
        theta_1 = |s|^2 / <s, dg> = 13/85  (the other quotient
        <s, dg> / |dg|^2 would give 85/733).
        beta = 1/2: x1 - (13/170) g1 = (63/136, 783/1360) >= 0,
        f = 22321741/3699200 ~ 6.0342 < fhat = 10: accepted.
    k = 2: g2 = (471/136, -1113/1360); s = (-39/136, 273/1360),
        dg = (s1, 9 s2); |s|^2 = 226629/1849600, <s, dg> = 822861/1849600,
        theta_2 = 149/541.  beta = 1/2: first component
        63/136 - (149/1082)(471/136) < 0 is clipped,
        x3 = (0, 1013043/1471520), f = 19497573089521/4330742220800 ~ 4.50213:
        accepted.
    k = 3: g3 = (3, 288267/1471520); s = (-63/136, 165837/1471520),
        theta_3 = (s1^2 + s2^2)/(s1^2 + 9 s2^2) = 1116014209/1614915081.
        beta = 1/2: x4 = (0, 983415589605721/1584253226662080) ~ (0, 0.62074),
        f(x4) ~ 4.50949 -- larger than f(x3) ~ 4.50213 (the step overshoots
        x2* = 2/3).  g3.(x3 - x4) ~ 0.013260.  The window of K = 2 gives
        fhat = max{f(x3), f(x2), f(x1)} = 949/128, and
        4.50949 < 949/128 - 0.25 * 0.013260 ~ 7.4107: accepted.  A monotone
        test (fhat = f(x3)) would reject it: 4.50949 >= 4.50213 - 0.00332.

    Totals after four iterations: 4 gradient and 6 function evaluations.
    """
    A = np.diag([1.0, 3.0])
    b = np.array([-3.0, 2.0])
    x0 = np.array([1.0, 0.0]).reshape(1, 1, 2)
    x, info, h = oracle.solve_dense(A, b, (1, 1, 2), x0=x0, hist_len=4, method=oracle.GPBB,
                                    alpha=0.0, tau=1e-4, eps=0.0, max_iter=4, gpbb_K=2,
                                    gpbb_sigma=0.25, gpbb_beta0=0.5)
    assert info["status"] == oracle.NOTCONV
    assert (info["iters"], info["grad_evals"], info["func_evals"]) == (4, 4, 6)
    # 1/theta_k for k = 0..3
    inv_theta = [1.0, 85.0 / 13.0, 541.0 / 149.0, 1614915081.0 / 1116014209.0]
    np.testing.assert_allclose(h["L"], inv_theta, rtol=1e-14)
    # f(x^(k)) for k = 0..3, and f(x^(4)) of the returned point
    f_k = [10.0, 949.0 / 128.0, 22321741.0 / 3699200.0, 19497573089521.0 / 4330742220800.0]
    np.testing.assert_allclose(h["phi"], f_k, rtol=1e-14)
    assert info["phi"] == pytest.approx(
        2515151318398222257764614588401 / 557746285819824850706335539200, rel=1e-14)
    assert x.ravel()[0] == 0.0
    assert x.ravel()[1] == pytest.approx(983415589605721 / 1584253226662080, rel=1e-14)


def _upn_run(L_bar, rho_L):
    g = synth.cone_geometry(6, 5, 9, 9, 1.5, 24.0, 36.0)
    x_true = synth.ellipsoid_phantom(6, 3, 7)
    b = oracle.noisy_data(g, x_true, synth.unit_noise(g.proj_shape, 8), 0.01)
    K = 60
    _, info, h = oracle.solve(g, b, method=oracle.UPN, alpha=1e-2, tau=1e-4, eps=0.0,
                              max_iter=K, hist_len=K, L_bar=L_bar, rho_L=rho_L)
    assert info["iters"] == K
    return h["L"], h["mu"], h["theta"]


@pytest.mark.parametrize("L_bar,rho_L", [(1.0, 2.0), (1e-2, 1.3)])
def test_upn_theta_solves_alg3_quadratic_with_current_mu_and_L(L_bar, rho_L):
    """Alg. 3: theta_{k+1} is the positive root of
    theta^2 = (1 - theta) theta_k^2 + (mu_k / L_k) theta, with the mu_k and
    L_k of iteration k, and theta_1 = sqrt(mu_0 / L_0).  History entry k holds
    L_k, mu_k and theta_{k+1}.  The run is one where L grows after the start
    (BT) and mu falls (eq. 9), so mu_k / L_k and mu_{k-1} / L_{k-1} differ and
    a root taken with the previous ratio leaves a residual of order 1e-2."""
    L, mu, th = _upn_run(L_bar, rho_L)
    K = len(L)
    q = mu / L
    assert np.all(np.diff(L) >= 0) and np.all(np.diff(mu) <= 0)
    assert any(L[k] > L[k - 1] for k in range(2, K)), "L must change after the start"
    assert sum(mu[k] < mu[k - 1] for k in range(2, K)) >= 5, "mu must change"
    assert th[0] == pytest.approx(np.sqrt(mu[0] / L[0]), rel=1e-15)
    assert np.all(th > 0.0) and np.all(th <= 1.0)
    res = np.array([th[k] ** 2 - (1.0 - th[k]) * th[k - 1] ** 2 - q[k] * th[k]
                    for k in range(1, K)])
    assert np.max(np.abs(res)) <= 1e-14
    # the check has teeth on this run: the previous iteration's ratio misses
    prev = np.array([th[k] ** 2 - (1.0 - th[k]) * th[k - 1] ** 2 - q[k - 1] * th[k]
                     for k in range(1, K)])
    assert np.max(np.abs(prev)) > 1e-3
