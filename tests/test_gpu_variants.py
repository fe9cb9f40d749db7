"""GPU parity of the method variants (Sec. III): Nesterov's method for given
mu and L, and a box Q = [lower, upper]^N.

* FP64: Nesterov and GP / UPN / GPBB under a box take the oracle's steps
  (same L sequence, iterates within 1e-9 after 25 iterations) and stay in
  the box.
* The batched solve (FP32) equals the single solve bit for bit for Nesterov
  and for boxed GP / UPN problems.
* Bad parameters are rejected.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")
DEV = "cuda"
BOX = (0.05, 0.8)


@pytest.fixture(scope="module")
def small():
    w = synth.cfg_small_parallel()
    og = oracle.Geometry(w.geom)
    b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
    # a safe L for Nesterov: twice the largest BT estimate of a UPN run
    _, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=1e-4,
                             max_iter=500, hist_len=500, bt_form=1)
    L = 2.0 * float(np.nanmax(ho["L"]))
    return w, og, b, L


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        DEV, torch.float64 if prec == tv.F64 else torch.float32)


def test_nesterov_steps_match_oracle_fp64(small):
    w, og, b, L = small
    mu = 1e-3 * L
    K = 25
    xo, io, ho = oracle.solve(og, b, method=oracle.NESTEROV, alpha=w.alpha, tau=w.tau, eps=0.0,
                              max_iter=K, hist_len=K, L_bar=L, mu_bar=mu, bt_form=1)
    G = tv.Geometry(w.geom, tv.F64)
    x, info, h = tv.solve(G, dev(b, tv.F64), method=tv.NESTEROV, alpha=w.alpha, tau=w.tau,
                          eps=0.0, max_iter=K, hist_len=K, L_bar=L, mu_bar=mu)
    assert info["iters"] == io["iters"] == K
    assert info["func_evals"] == K  # no line-search trials beyond the one step
    np.testing.assert_array_equal(np.array(h["L"]), np.full(K, L))
    assert abs(info["mu"] - mu) == 0.0
    assert np.max(np.abs(x.cpu().numpy() - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)


@pytest.mark.parametrize("method", ["gp", "upn", "gpbb"])
def test_box_steps_match_oracle_fp64(small, method):
    w, og, b, _ = small
    tm, om = {"gp": (tv.GP, oracle.GP), "upn": (tv.UPN, oracle.UPN),
              "gpbb": (tv.GPBB, oracle.GPBB)}[method]
    K = 25
    xo, io, ho = oracle.solve(og, b, method=om, alpha=w.alpha, tau=w.tau, eps=0.0, max_iter=K,
                              hist_len=K, bt_form=1, lower=BOX[0], upper=BOX[1])
    G = tv.Geometry(w.geom, tv.F64)
    x, info, h = tv.solve(G, dev(b, tv.F64), method=tm, alpha=w.alpha, tau=w.tau, eps=0.0,
                          max_iter=K, hist_len=K, lower=BOX[0], upper=BOX[1])
    assert info["iters"] == io["iters"]
    n = len(h["L"])
    np.testing.assert_allclose(np.array(h["L"]), ho["L"][:n], rtol=1e-9 if method == "gpbb"
                               else 0, atol=0)
    xg = x.cpu().numpy()
    assert xg.min() >= BOX[0] and xg.max() <= BOX[1]
    assert np.max(np.abs(xg - xo)) <= 1e-9 * max(np.max(np.abs(xo)), 1.0)


def test_batched_variants_equal_single(small):
    w, og, b, L = small
    bd = dev(b, tv.F32)
    base = dict(alpha=w.alpha, tau=w.tau, eps=1e-4, max_iter=300)
    params = [dict(base, method=tv.NESTEROV, L_bar=L, mu_bar=1e-3 * L),
              dict(base, method=tv.UPN, lower=BOX[0], upper=BOX[1]),
              dict(base, method=tv.GP, lower=-0.5, upper=0.5),
              dict(base, method=tv.UPN)]
    geoms = [tv.Geometry(w.geom, tv.F32) for _ in params]
    singles = [tv.solve(G, bd, **p) for G, p in zip(geoms, params)]
    xb, ib, _ = tv.solve_batched(geoms, [bd] * len(params), params)
    for i, (x, info, _) in enumerate(singles):
        assert torch.equal(xb[i], x), i
        assert ib[i]["iters"] == info["iters"], i
    assert float(xb[1].min()) >= BOX[0] and float(xb[1].max()) <= BOX[1]
    assert float(xb[2].min()) >= -0.5 and float(xb[2].max()) <= 0.5


@pytest.mark.parametrize("bad", [dict(method=3, L_bar=1.0, mu_bar=2.0),
                                 dict(method=3, L_bar=float("inf"), mu_bar=0.0),
                                 dict(lower=0.5, upper=0.5), dict(lower=1.0, upper=0.0),
                                 dict(lower=float("nan"), upper=1.0)])
def test_bad_variant_parameters_rejected(small, bad):
    w, og, b, _ = small
    G = tv.Geometry(w.geom, tv.F32)
    with pytest.raises(tv.TvregError):
        tv.solve(G, dev(b, tv.F32), max_iter=5, **bad)
