"""UPN on the 64^3 cone-beam workload (20 views of 96 x 96 at pitch 1.5,
R = 256, SDD = 384, 1 % noise, alpha 1e-3 and 1e-2) against the FP64 oracle,
step by step over the first 25 iterations from x0 = 0:

* FP64: the same line-search decisions (L sequence) and iterates within 1e-9
  of the oracle's scale;
* FP32 storage with FP64 reductions: the same L sequence, and iterates within
  2e-5 of the oracle's scale (FP32 rounding of the vectors, amplified by the
  momentum steps; measured 1.1e-6 and 8.6e-7; FP64 3.4e-14).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")
K = 25


@pytest.fixture(scope="module", params=[1e-3, 1e-2])
def run(request):
    w = synth.cfg_cone64(request.param)
    og = oracle.Geometry(w.geom)
    b = oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)
    print(f"cone64 alpha={w.alpha}: oracle UPN, {K} iterations", flush=True)
    xo, io, ho = oracle.solve(og, b, method=oracle.UPN, alpha=w.alpha, tau=w.tau, eps=0.0,
                              max_iter=K, hist_len=K, bt_form=1)
    return w, b, xo, io, ho


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
def test_cone64_upn_steps_match_oracle(run, prec):
    w, b, xo, io, ho = run
    dt = torch.float64 if prec == tv.F64 else torch.float32
    G = tv.Geometry(w.geom, prec)
    x, info, h = tv.solve(G, torch.from_numpy(b).to("cuda", dt), method=tv.UPN,
                          alpha=w.alpha, tau=w.tau, eps=0.0, max_iter=K, hist_len=K)
    assert info["iters"] == io["iters"] == K
    np.testing.assert_array_equal(np.array(h["L"]), ho["L"][:K])
    err = np.max(np.abs(x.cpu().double().numpy() - xo)) / np.max(np.abs(xo))
    print(f"cone64 alpha={w.alpha} prec={prec}: max rel err {err:.3e}", flush=True)
    assert err <= (1e-9 if prec == tv.F64 else 2e-5)
