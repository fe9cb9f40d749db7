"""GPU checks of the batched GP / UPN solve (tvreg_solve_batched).

The batched driver runs the single-problem kernels' per-block work inside
grouped launches and takes each problem's line-search, mu and stop decisions
in a device control kernel with the same double arithmetic as tvreg_solve.
So the bar is bit-for-bit: every problem's result and every reported scalar
must equal what tvreg_solve returns for that problem alone (tvreg_solve is
itself held to the FP64 oracle by the solver parity tests).  Covered: mixed
GP / UPN, cone and parallel, ragged sizes, per-problem alpha, a start point
with negative entries (clipped), a stop at the first iteration, a stall in
the first line search, the iteration cap, and the poll interval.
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


def mixed_problems():
    """(geometry, data seed, solve kwargs, start-point kind) per problem."""
    return [
        (synth.cfg_small_parallel().geom, 11,
         dict(method=tv.UPN, alpha=1e-2, eps=1e-5, max_iter=300), "zero"),
        (synth.Geometry(37, 29, 23, synth.view_angles(7, 2 * math.pi), synth.CONE, 41, 19, 2.1,
                        2.3, 60.0, 110.0), 12,
         dict(method=tv.UPN, alpha=3e-3, eps=1e-3, max_iter=40), "zero"),
        (synth.Geometry(37, 29, 23, synth.view_angles(5, math.pi), synth.PARALLEL, 43, 23, 1.0,
                        1.0), 13,
         dict(method=tv.GP, alpha=1e-2, eps=1e-9, max_iter=25), "zero"),
        (synth.Geometry(8, 8, 8, np.array([0.2, 2.0, 4.1]), synth.CONE, 12, 12, 1.5, 1.5, 32.0,
                        48.0), 14,
         dict(method=tv.UPN, alpha=1e-2, eps=1.0, max_iter=50), "zero"),       # stops at once
        (synth.Geometry(1, 1, 1, np.array([0.3]), synth.CONE, 3, 3, 1.5, 1.5, 4.0, 6.0), 15,
         dict(method=tv.UPN, alpha=1e-2, eps=1e-6, max_iter=50, L_bar=1e-12, max_trials=3),
         "random"),                                                              # stalls
        (synth.Geometry(6, 9, 7, np.array([0.4, 1.7, 3.3, 5.0]), synth.CONE, 16, 11, 1.3, 1.2,
                        30.0, 50.0), 16,
         dict(method=tv.UPN, alpha=1e-2, eps=1e-8, max_iter=60), "signed"),    # clipped start
        (synth.cone_geometry(12, 8, 18, 16, 1.5, 48.0, 72.0), 17,
         dict(method=tv.UPN, alpha=1e-2, eps=1e-6, max_iter=80), "zero"),      # quarter turns + mirror
    ]


def make_inputs(geom, seed, start, prec):
    og = oracle.Geometry(geom)
    shape = (geom.nz, geom.ny, geom.nx)
    b = oracle.noisy_data(og, synth.random_volume(shape, seed),
                          synth.unit_noise(geom.proj_shape, seed + 100), 0.01)
    if start == "zero":
        x0 = np.zeros(shape)
    elif start == "random":
        x0 = synth.random_volume(shape, seed + 200)
    else:
        x0 = synth.random_volume(shape, seed + 200, -0.5, 1.0)
    return dev(b, prec), dev(x0, prec)


def single_kwargs(kw):
    k = dict(kw)
    k.setdefault("L_bar", 1.0)
    k.setdefault("max_trials", 60)
    return k


def run_both(problems, prec, poll=8, tau=1e-4):
    geoms, bs, x0s, kws = [], [], [], []
    for geom, seed, kw, start in problems:
        geoms.append(tv.Geometry(geom, prec))
        b, x0 = make_inputs(geom, seed, start, prec)
        bs.append(b)
        x0s.append(x0)
        kws.append(single_kwargs(kw))
    singles = []
    for G, b, x0, kw in zip(geoms, bs, x0s, kws):
        x, info, _ = tv.solve(G, b, tau=tau, x0=x0, **kw)
        singles.append((x, info))
    return geoms, bs, x0s, kws, singles


def batched(geoms, bs, x0s, kws, poll, tau=1e-4):
    return tv.solve_batched(geoms, bs, [dict(k, tau=tau) for k in kws], x0s=x0s,
                            poll_rounds=poll)


def assert_same(xb, ib, xs, is_, what):
    assert torch.equal(xb, xs), f"{what}: x differs, max {float((xb - xs).abs().max()):.3e}"
    for k in ("iters", "grad_evals", "func_evals", "stop_reason"):
        assert ib[k] == is_[k], f"{what}: {k} {ib[k]} vs {is_[k]}"
    for k in ("phi", "gm_rel", "gm_abs_over_N", "L", "mu"):
        a, c = ib[k], is_[k]
        assert (math.isnan(a) and math.isnan(c)) or a == c, f"{what}: {k} {a!r} vs {c!r}"


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
@pytest.mark.parametrize("poll", [1, 8])
def test_batched_equals_single_solves(prec, poll):
    print(f"batch vs single prec={prec} poll={poll}", flush=True)
    probs = mixed_problems()
    geoms, bs, x0s, kws, singles = run_both(probs, prec)
    # GP and UPN problems in one batch
    xb, ib, status = batched(geoms, bs, x0s, kws, poll)
    for i in range(len(probs)):
        assert_same(xb[i], ib[i], singles[i][0], singles[i][1], f"problem {i}")
    reasons = [i["stop_reason"] for i in ib]
    expect = tv.ESTALL if tv.ESTALL in reasons else (
        tv.ENOTCONV if tv.ENOTCONV in reasons else tv.OK)
    assert status == expect
    # the cases the batch was built to cover did occur
    reasons = [s[1]["stop_reason"] for s in singles]
    assert singles[3][1]["iters"] == 1 and reasons[3] == tv.OK
    assert reasons[4] == tv.ESTALL
    assert reasons[2] == tv.ENOTCONV
    assert torch.equal(singles[4][0], x0s[4].clamp_min(0))


# (projector tile columns, waves per block, backprojector depth), one per
# problem of mixed_problems(): every block height and both tile kinds appear
TUNED_SHAPES = [(1, 2, 4), (8, 8, 16), (2, 1, 8), (64, 8, 4), (16, 1, 16), (32, 2, 4),
                (2, 4, 8)]


@pytest.mark.parametrize("prec", [tv.F64, tv.F32])
def test_batched_equals_single_solves_under_tuned_shapes(prec):
    """Each problem of a batch runs its own geometry's tile shapes (the
    grouped projector is launched once per block shape, each problem with
    its own tile width; the grouped backprojector takes each problem's
    depth), so the batch still equals the single solves bit for bit."""
    print(f"batch vs single, tuned shapes, prec={prec}", flush=True)
    probs = mixed_problems()
    geoms, bs, x0s, kws = [], [], [], []
    for (geom, seed, kw, start), shape in zip(probs, TUNED_SHAPES):
        G = tv.Geometry(geom, prec)
        G.set_tuning(*shape)
        assert G.tuning == shape
        geoms.append(G)
        b, x0 = make_inputs(geom, seed, start, prec)
        bs.append(b)
        x0s.append(x0)
        kws.append(single_kwargs(kw))
    singles = [tv.solve(G, b, tau=1e-4, x0=x0, **kw)[:2]
               for G, b, x0, kw in zip(geoms, bs, x0s, kws)]
    xb, ib, _ = batched(geoms, bs, x0s, kws, 8)
    for i in range(len(probs)):
        assert_same(xb[i], ib[i], singles[i][0], singles[i][1], f"problem {i}")


def test_batched_start_point_untouched_and_inputs_reusable():
    probs = mixed_problems()[:2]
    geoms, bs, x0s, kws, singles = run_both(probs, tv.F32)
    keep = [x.clone() for x in x0s]
    xb, ib, _ = batched(geoms, bs, x0s, kws, 8)
    for a, c in zip(x0s, keep):
        assert torch.equal(a, c)
    xb2, ib2, _ = batched(geoms, bs, x0s, kws, 3)
    for j in range(2):
        assert torch.equal(xb[j], xb2[j])
        assert ib[j] == ib2[j]


def test_batched_rejects_bad_arguments():
    g = tv.Geometry(synth.cfg_small_parallel().geom, tv.F32)
    g64 = tv.Geometry(synth.cfg_small_parallel().geom, tv.F64)
    b = torch.zeros(g.proj_shape, device=DEV)
    with pytest.raises(tv.TvregError) as e:  # GPBB is not batched
        tv.solve_batched([g], [b], [dict(method=tv.GPBB)])
    assert e.value.status == tv.EINVAL
    with pytest.raises(tv.TvregError) as e:
        tv.solve_batched([g], [b], [dict(rho_L=1.0)])
    assert e.value.status == tv.EINVAL
    with pytest.raises(ValueError):  # mixed precisions
        tv.solve_batched_workspace([g, g64])
    with pytest.raises(ValueError):
        tv.solve_batched([g], [b], [dict(gpbb_K=3)])
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    with pytest.raises(tv.TvregError) as e:
        tv.solve_batched([g], [b], [{}], workspace=ws)
    assert e.value.status == tv.ENOMEM


def test_batch_workload_sampled_problems_match_single_solves():
    """The 32-problem batch of uneven sizes (n in 32..128, 10-40 views, alpha
    1e-4..1e-1), F32 with FP64 reductions: three sampled problems (smallest,
    largest, first) equal their own tvreg_solve bit for bit, and every
    problem converges.  Data from the FP64 projector of the library (the
    check is library against library; both sides read the same b)."""
    ws_ = synth.cfg_batch()
    prec = tv.F32
    geoms, bs, kws = [], [], []
    for w in ws_:
        G64 = tv.Geometry(w.geom, tv.F64)
        ax = tv.project(G64, dev(w.phantom(), tv.F64))
        sigma = w.eta * float(torch.linalg.norm(ax)) / math.sqrt(ax.numel())
        b = ax + sigma * dev(w.unit_noise(), tv.F64)
        del G64
        geoms.append(tv.Geometry(w.geom, prec))
        bs.append(b.float().contiguous())
        kws.append(dict(method=tv.UPN, alpha=w.alpha, eps=1e-4, max_iter=2000, L_bar=1.0,
                        max_trials=60))
    print("batch32 solving", flush=True)
    xb, ib, status = batched(geoms, bs, None, kws, 8)
    assert status == tv.OK, [i["stop_reason"] for i in ib]
    sizes = [g.N for g in geoms]
    for i in sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0}):
        x, info, _ = tv.solve(geoms[i], bs[i], tau=1e-4, **kws[i])
        assert_same(xb[i], ib[i], x, info, f"batch problem {i}")
