"""GPU parity of the differentiated form (unrolled UPN and its reverse pass)
against the FP64 oracle, plus the TV Hessian-vector stencil it relies on.

* tvreg_tv_hessvec: FP64 within 1e-12 of the oracle (relative to the
  output's scale), FP32 per element within its own rounding plus a small
  scale-relative allowance, on volumes that span several tiles with ragged
  edges and on both smoothing regimes.
* FP64 unrolled forward: the line-search decisions equal the oracle's and
  x^(K) agrees to 1e-10; the reverse pass agrees to 1e-8 in dl/dlog(alpha)
  and in dl/db (relative L2).
* FP32 with FP64 reductions, the oracle's L_j replayed, both sides reading
  the same FP32 values of b and x_true: x^(K) within 1e-4 relative L2 and
  both gradients within 1e-3 (the map amplifies rounding by the Jacobian of
  the unrolled steps, gain ~10 here), or within 4x the oracle gradient's own
  sensitivity to FP32 roundoff of b where that is larger (the small
  tau = 1e-4 case).  At 64^3 the FP32 path's own line search also takes
  the oracle's decisions.
* Checkpoint spacing does not change a single bit of the gradients.
* torch.autograd: the Function's gradient matches central differences of its
  own forward pass (FP64, decisions replayed).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")
DEV = "cuda"


def dev(a, prec):
    return torch.from_numpy(np.ascontiguousarray(a)).to(
        DEV, torch.float64 if prec == tv.F64 else torch.float32)


def host(t):
    return t.detach().cpu().double().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def forward_diffs(a):
    d = []
    for ax in (2, 1, 0):
        e = np.zeros_like(a)
        sl = [slice(None)] * 3
        sl[ax] = slice(0, -1)
        e[tuple(sl)] = np.diff(a, axis=ax)
        d.append(e)
    return d


def term_scale(y, v, tau):
    dy = forward_diffs(y)
    dv = forward_diffs(v)
    ny = np.sqrt(sum(c * c for c in dy))
    nv = np.sqrt(sum(c * c for c in dv))
    return float(np.max(nv / np.maximum(ny, tau)))


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("shape,tau", [((23, 37, 70), 1e-4), ((17, 9, 130), 0.3),
                                       ((40, 41, 67), 10.0), ((1, 1, 5), 1e-4)])
def test_hessvec_matches_oracle(prec, shape, tau):
    print(f"hessvec {shape} tau={tau} prec={prec}", flush=True)
    y = synth.random_volume(shape, 31)
    v = synth.random_volume(shape, 32, -1.0, 1.0)
    if prec == tv.F32:
        y = y.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    ref = oracle.tv_hessvec(y, v, tau)
    _, g = oracle.tv(y, tau)
    dot_ref = float(np.sum(v * g))
    out, dot = tv.tv_hessvec(dev(y, prec), dev(v, prec), tau)
    got = host(out)
    # errors scale with the per-voxel terms |D_j v| / max(tau, |D_j y|), which
    # can cancel to an exactly zero Hessian (a 1-D profile in the linear regime)
    scale = max(np.max(np.abs(ref)), term_scale(y, v, tau))
    if prec == tv.F64:
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale
        assert abs(float(dot) - dot_ref) <= 1e-12 * max(abs(dot_ref), 1.0)
    else:
        # per-voxel terms in float: a few roundings of the largest term
        assert np.max(np.abs(got - ref)) <= 2e-6 * scale
        assert abs(float(dot) - dot_ref) <= 1e-5 * max(np.sum(np.abs(v * g)), 1.0)


def small_problem():
    # even detector: no pixel centre at u = 0, whose ray at theta = pi would
    # run 1e-16 off the y = 0 voxel face (ill-posed for any two implementations)
    n = 10
    geom = synth.cone_geometry(n, 6, 16, 16, 1.5, 4 * n, 6 * n)
    og = oracle.Geometry(geom)
    xt = synth.ellipsoid_phantom(n, 4, 7)
    b = oracle.noisy_data(og, xt, synth.unit_noise(og.proj_shape, 8), 0.01)
    return geom, og, xt, b


def cfg5_problem():
    w = synth.cfg_unrolled()
    og = oracle.Geometry(w.geom)
    xt = w.phantom()
    b = oracle.noisy_data(og, xt, w.unit_noise(), w.eta)
    return w.geom, og, xt, b, w.alpha, w.tau


def gpu_grad(G, b, xt, K, alpha, tau, prec, ckpt=5, L_replay=None):
    bd = dev(b, prec)
    xK, tape, L = tv.upn_unrolled_fwd(G, bd, K, alpha, tau=tau, ckpt_every=ckpt,
                                      L_replay=L_replay)
    xb = 2.0 * (xK - dev(xt, prec))
    da, db = tv.upn_unrolled_bwd(G, bd, tape, xb)
    return xK, L, da, db


@pytest.mark.parametrize("K,alpha,tau", [(30, 1e-2, 1e-2), (10, 1e-2, 1e-4), (30, 1e-2, 1e-4)])
def test_unrolled_fp64_matches_oracle(K, alpha, tau):
    print(f"unrolled fp64 K={K} alpha={alpha} tau={tau}", flush=True)
    geom, og, xt, b = small_problem()
    o = oracle.unrolled(og, b, K, alpha, tau=tau)
    og_g = oracle.unrolled(og, b, K, alpha, tau=tau, L=o["L"], xK_bar=2.0 * (o["xK"] - xt))
    G = tv.Geometry(geom, tv.F64)
    xK, L, da, db = gpu_grad(G, b, xt, K, alpha, tau, tv.F64)
    np.testing.assert_array_equal(np.array(L), o["L"])
    assert rel(host(xK), o["xK"]) <= 1e-10
    assert abs(da - alpha * og_g["alpha_bar"]) <= 1e-8 * abs(alpha * og_g["alpha_bar"])
    assert rel(host(db), og_g["b_bar"]) <= 1e-8


def fp32_sensitivity(og, b, xt, K, alpha, tau, L, g0):
    """How far the exact (FP64) gradient moves when b moves by FP32 unit
    roundoff (2^-24, relative, seeded direction): the resolution any FP32
    evaluation of this gradient can be held to."""
    u = 2.0 ** -24
    bp = b * (1.0 + u * synth.unit_noise(b.shape, 77))
    o2 = oracle.unrolled(og, bp, K, alpha, tau=tau, L=L)
    g = oracle.unrolled(og, bp, K, alpha, tau=tau, L=L, xK_bar=2.0 * (o2["xK"] - xt))
    da = abs(g["alpha_bar"] - g0["alpha_bar"]) / abs(g0["alpha_bar"])
    db = rel(g["b_bar"], g0["b_bar"])
    return da, db


def as_f32(a):
    """The FP32 path reads b and x_true as float values; the oracle is given
    those same values (input rounding is not a precision error)."""
    return np.asarray(a, np.float32).astype(np.float64)


# Both sides read the same FP32 values of b and x_true.  At tau = 1e-4 the
# unrolled map's Jacobian varies fast (voxels near the Huber kink, where the
# TV Hessian is up to 1/tau): a relative change of b at FP32 roundoff (2^-24)
# moves the exact gradient by ~1e-2 on this 10^3 problem, and the FP32 path
# rounds every iterate at that level, so it is held to 4x the oracle's own
# sensitivity at FP32 roundoff (and to 1e-3 where that is larger).
@pytest.mark.parametrize("K,alpha,tau", [(30, 1e-2, 1e-2), (30, 1e-2, 1e-4)])
def test_unrolled_fp32_matches_oracle(K, alpha, tau):
    print(f"unrolled fp32 K={K} alpha={alpha} tau={tau}", flush=True)
    geom, og, xt, b = small_problem()
    xt, b = as_f32(xt), as_f32(b)
    o = oracle.unrolled(og, b, K, alpha, tau=tau)
    og_g = oracle.unrolled(og, b, K, alpha, tau=tau, L=o["L"], xK_bar=2.0 * (o["xK"] - xt))
    sa, sb = fp32_sensitivity(og, b, xt, K, alpha, tau, o["L"], og_g)
    G = tv.Geometry(geom, tv.F32)
    xK, L, da, db = gpu_grad(G, b, xt, K, alpha, tau, tv.F32, L_replay=list(o["L"]))
    ref_a = alpha * og_g["alpha_bar"]
    ea, eb = abs(da - ref_a) / abs(ref_a), rel(host(db), og_g["b_bar"])
    print(f"  alpha-grad err {ea:.2e} (sensitivity {sa:.2e}), b-grad err {eb:.2e} "
          f"(sensitivity {sb:.2e})", flush=True)
    assert rel(host(xK), o["xK"]) <= 1e-4
    assert ea <= max(1e-3, 4.0 * sa)
    assert eb <= max(1e-3, 4.0 * sb)


def test_unrolled_64cube_30views_fp32_matches_oracle():
    """The differentiated workload at full size: 64^3, cone beam, 30 views,
    96 x 96 detector, K = 30 (the oracle's BT decisions replayed)."""
    geom, og, xt, b, alpha, tau = cfg5_problem()
    xt, b = as_f32(xt), as_f32(b)
    K = 30
    print("unrolled 64^3 oracle", flush=True)
    o = oracle.unrolled(og, b, K, alpha, tau=tau)
    assert o["status"] == 0
    og_g = oracle.unrolled(og, b, K, alpha, tau=tau, L=o["L"], xK_bar=2.0 * (o["xK"] - xt))
    print("unrolled 64^3 gpu", flush=True)
    G = tv.Geometry(geom, tv.F32)
    xK, L, da, db = gpu_grad(G, b, xt, K, alpha, tau, tv.F32, L_replay=list(o["L"]))
    ref_a = alpha * og_g["alpha_bar"]
    print(f"64^3 K=30: x rel {rel(host(xK), o['xK']):.2e}  dl/dlog(alpha) rel "
          f"{abs(da - ref_a) / abs(ref_a):.2e}  dl/db rel {rel(host(db), og_g['b_bar']):.2e}",
          flush=True)
    assert rel(host(xK), o["xK"]) <= 1e-4
    assert abs(da - ref_a) <= 1e-3 * abs(ref_a), (da, ref_a)
    assert rel(host(db), og_g["b_bar"]) <= 1e-3
    # the FP32 path's own line search (no replay) takes the oracle's decisions
    _, L32, _, _ = gpu_grad(G, b, xt, K, alpha, tau, tv.F32)
    np.testing.assert_array_equal(np.array(L32), o["L"])


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
def test_checkpoint_spacing_is_bit_exact(prec):
    geom, og, xt, b = small_problem()
    G = tv.Geometry(geom, prec)
    ref = None
    for ck in (1, 5, 7, 30):
        xK, L, da, db = gpu_grad(G, b, xt, 30, 1e-2, 1e-4, prec, ckpt=ck)
        if ref is None:
            ref = (xK, da, db)
        else:
            assert torch.equal(xK, ref[0])
            assert da == ref[1]
            assert torch.equal(db, ref[2])


def test_autograd_function_matches_central_differences():
    geom, og, xt, b = small_problem()
    G = tv.Geometry(geom, tv.F64)
    K, tau = 30, 1e-2
    bd = dev(b, tv.F64)
    xtd = dev(xt, tv.F64)
    la = torch.tensor(math.log(1e-2), dtype=torch.float64, device=DEV, requires_grad=True)
    bv = bd.clone().requires_grad_(True)
    _, _, L = tv.upn_unrolled_fwd(G, bd, K, 1e-2, tau=tau)

    def loss(bb, a):
        x = tv.unrolled_upn(G, bb, a, K=K, tau=tau, L_replay=L)
        return ((x - xtd) ** 2).sum()

    l0 = loss(bv, la)
    l0.backward()
    h = 1e-6
    with torch.no_grad():
        lp = float(loss(bd, la.detach() + h))
        lm = float(loss(bd, la.detach() - h))
    fd_a = (lp - lm) / (2 * h)
    assert abs(float(la.grad) - fd_a) <= 1e-6 * abs(fd_a)
    w = dev(synth.fd_direction(og.proj_shape, 503), tv.F64)
    e = h * float(torch.sqrt(torch.mean(bd * bd)))
    with torch.no_grad():
        lp = float(loss(bd + e * w, la.detach()))
        lm = float(loss(bd - e * w, la.detach()))
    fd_b = (lp - lm) / (2 * e)
    ad_b = float(torch.sum(bv.grad * w))
    assert abs(ad_b - fd_b) <= 1e-6 * abs(fd_b)


def test_unrolled_stall_and_bad_arguments():
    geom, og, xt, b = small_problem()
    G = tv.Geometry(geom, tv.F32)
    bd = dev(b, tv.F32)
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_fwd(G, bd, 0, 1e-2, tape=tv.unrolled_workspace(G, 3, 5))
    assert e.value.status == tv.EINVAL
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_fwd(G, bd, 3, 1e-2, L_replay=[1.0, -1.0, 1.0])
    assert e.value.status == tv.EINVAL
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_fwd(G, bd, 3, 1e-2, tape=torch.empty(64, dtype=torch.uint8, device=DEV))
    assert e.value.status == tv.ENOMEM
    xK, tape, L = tv.upn_unrolled_fwd(G, bd, 3, 1e-2)
    # a stalled line search (one trial allowed, L_bar far too small) leaves no gradient
    t2 = tv.unrolled_workspace(G, 3, 5)
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_fwd(G, bd, 3, 1e-2, L_bar=1e-9, max_trials=1, tape=t2)
    assert e.value.status == tv.ESTALL
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_bwd(G, bd, t2, torch.zeros_like(xK))
    assert e.value.status == tv.EINVAL
    # a tape written for another geometry is refused
    w = synth.cfg_small_parallel().geom
    G2 = tv.Geometry(w, tv.F32)
    with pytest.raises(tv.TvregError) as e:
        tv.upn_unrolled_bwd(G2, dev(np.zeros(w.proj_shape), tv.F32), tape,
                            torch.zeros(w.vol_shape, device=DEV))
    assert e.value.status == tv.EINVAL


def test_unrolled_rejects_other_methods_and_boxes():
    """The differentiated form is UPN over the orthant: other methods and a
    box are refused through the C ABI rather than ignored."""
    import ctypes
    geom, og, xt, b = small_problem()
    G = tv.Geometry(geom, tv.F32)
    bd = dev(b, tv.F32)
    tape = tv.unrolled_workspace(G, 3, 5)
    xK = G.empty_volume()
    for method, box in ((tv.GP, (0, 0.0, 0.0)), (tv.NESTEROV, (0, 0.0, 0.0)),
                        (tv.UPN, (1, 0.0, 1.0))):
        p = tv._SolveParams(method, 1e-2, 1e-4, 0.0, 0, 1, 1.0, 0.0, 2.0, 2, 0.1, 0.95, 60,
                            None, None, None, 0, *box)
        st = tv.lib().tvreg_upn_unrolled_fwd(G.handle, ctypes.c_void_p(bd.data_ptr()),
                                             ctypes.byref(p), 3, 5, None, None,
                                             ctypes.c_void_p(xK.data_ptr()),
                                             ctypes.c_void_p(tape.data_ptr()), tape.numel(),
                                             None)
        assert st == tv.EINVAL, (method, box)
