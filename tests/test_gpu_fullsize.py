"""Full-size parity on the 256^3 cone-beam scan (60 views of 384 x 256), in
the launch configurations the benchmark times: FP32 vectors with FP64 sums,
tile shapes chosen by the autotuner, and the backprojector either on the fly
through the scan's symmetry (the headline's) or from the stored A^T.  The
data b comes from the oracle (its projection of the phantom plus the seeded
noise).

* phi and grad phi at the phantom against the oracle's FP64 evaluation at the
  same FP32 values: phi within 1e-6 relative; every gradient element within
  the FP32 rounding of its data part plus a 2e-6 allowance relative to the
  gradient's scale (the FP32 TV stencil, as in the TV test at this size).
* Ten UPN, GPBB and GP iterations from x0 = 0: the iterate is feasible, and
  the objective the solver reports for it (an FP64 sum over its FP32
  residual and TV terms) matches the oracle's phi at the returned FP32
  iterate within 1e-6.
* The benchmark's solve run to convergence (UPN, FP32, 1e-6 relative
  gradient map; the oracle's own minimiser is hours away on the host): the
  oracle certifies the returned iterate, its FP64 gradient map there
  |G_L(x)| (nu = the final L; eq. 10) relative to |G(x0 = 0)| is at most
  2e-6, and the objective the solver reports is the oracle's phi at x within
  1e-6.  Both sides read b rounded to FP32.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")
DEV = "cuda"


@pytest.fixture(scope="module")
def data():
    w = synth.cfg_cone256()
    print("cone256: oracle data", flush=True)
    return w, oracle.noisy_data(w.geom, w.phantom(), w.unit_noise(), w.eta)


@pytest.fixture(scope="module", params=["on_the_fly", "stored"])
def scan(request, data):
    w, b = data
    G = tv.Geometry(w.geom, tv.F32)
    print(f"cone256: backprojector {request.param}; autotune", flush=True)
    if request.param == "stored":
        G.attach_matrix()
    t = G.autotune(reps=2)
    print(f"cone256: tuned {G.tuning}, projector {t['project_ms'][t['project_tile_cols'], t['project_waves']]:.3f} ms",
          flush=True)
    bd = torch.from_numpy(b).to(DEV, torch.float32)
    return w, b, G, bd


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def test_cone256_objective_grad_matches_oracle(scan):
    w, b, G, bd = scan
    x = f32(w.phantom())
    print("cone256: GPU phi / grad", flush=True)
    phi, g = tv.objective_grad(G, bd, w.alpha, w.tau, torch.from_numpy(x).to(DEV, torch.float32))
    got = g.cpu().double().numpy()
    print("cone256: oracle phi / grad", flush=True)
    phi_ref, g_ref = oracle.phi_grad(w.geom, b, w.alpha, w.tau, x)
    assert abs(float(phi.item()) - phi_ref) <= 1e-6 * abs(phi_ref)
    # data part A^T r: r rounded once to FP32, the stored values (if any)
    # rounded once, the sum in double; the output rounded once
    r = oracle.project(w.geom, x) - b.reshape(w.geom.proj_shape)
    data_bound = oracle.backproject(w.geom, np.abs(r))
    scale = np.max(np.abs(g_ref))
    tol = 2.0 ** -23 * data_bound + 2.0 ** -24 * np.abs(g_ref) + 2e-6 * scale
    bad = np.abs(got - g_ref) > tol
    assert not bad.any(), f"{bad.sum()} gradient entries off, worst {np.max(np.abs(got - g_ref)):.3e}"


@pytest.mark.parametrize("method", ["upn", "gpbb", "gp"])
def test_cone256_iterations_objective_matches_oracle(scan, method):
    w, b, G, bd = scan
    m = {"upn": tv.UPN, "gpbb": tv.GPBB, "gp": tv.GP}[method]
    print(f"cone256: 10 {method} iterations", flush=True)
    x, info, _ = tv.solve(G, bd, method=m, alpha=w.alpha, tau=w.tau, eps=0.0, max_iter=10)
    assert info["iters"] == 10
    xh = x.cpu().double().numpy()
    assert xh.min() >= 0.0
    print("cone256: oracle phi at the iterate", flush=True)
    phi_ref = oracle.phi(w.geom, b, w.alpha, w.tau, xh)
    phi0 = oracle.phi(w.geom, b, w.alpha, w.tau, np.zeros_like(xh))
    assert phi_ref < 0.5 * phi0
    assert abs(info["phi"] - phi_ref) <= 1e-6 * phi_ref, (info["phi"], phi_ref)


def test_cone256_upn_f32_to_tolerance_certified_by_oracle(scan):
    w, b, G, bd = scan
    b32 = f32(b)
    print("cone256: UPN f32 to 1e-6", flush=True)
    x, info, _ = tv.solve(G, bd, method=tv.UPN, alpha=w.alpha, tau=w.tau, eps=1e-6,
                          max_iter=5000)
    assert info["stop_reason"] == tv.OK
    assert info["gm_rel"] <= 1e-6
    xh = x.cpu().double().numpy()
    assert xh.min() >= 0.0
    print(f"cone256: converged after {info['iters']}; oracle gradient at x", flush=True)
    phi_ref, g_ref = oracle.phi_grad(w.geom, b32, w.alpha, w.tau, xh)
    print("cone256: oracle gradient at x0 = 0", flush=True)
    zero = np.zeros_like(xh)
    _, g0 = oracle.phi_grad(w.geom, b32, w.alpha, w.tau, zero)
    gm0 = oracle.gradmap_norm(zero, g0, 1.0)   # |min(grad f(0), 0)|, any nu
    gm = oracle.gradmap_norm(xh, g_ref, info["L"])
    print(f"cone256: oracle |G(x)|/|G(0)| = {gm / gm0:.3e} (solver {info['gm_rel']:.3e}); "
          f"phi {info['phi']:.10e} vs {phi_ref:.10e}", flush=True)
    assert gm / gm0 <= 2e-6
    assert abs(info["phi"] - phi_ref) <= 1e-6 * phi_ref
