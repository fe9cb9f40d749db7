"""A gradient evaluation (tvreg_objective_grad: transpose, projection,
backprojection, TV, finalisers; kernel launches only) captured in a HIP graph
gives, on every replay, bitwise the eager result -- with eager work and
synchronisations between the replays -- for the on-the-fly and the stored
operators."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

tv = pytest.importorskip("paper_1105_4002_amd")


@pytest.mark.parametrize("stored", [False, True])
def test_objective_grad_graph_replays_match_eager(stored):
    w = synth.cfg_cone64()
    og = oracle.Geometry(w.geom)
    b = torch.from_numpy(oracle.noisy_data(og, w.phantom(), w.unit_noise(), w.eta)).to(
        "cuda", torch.float32)
    G = tv.Geometry(w.geom, tv.F32)
    if stored:
        G.attach_matrix()
    x = torch.from_numpy(w.phantom()).to("cuda", torch.float32)
    ws = tv.objective_workspace(G)
    g_eager = G.empty_volume()
    phi_eager, _ = tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g_eager, workspace=ws)
    phi_eager = phi_eager.clone()
    g = G.empty_volume()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        phi_g, _ = tv.objective_grad(G, b, w.alpha, w.tau, x, grad=g, workspace=ws)
    for rep in range(4):
        g.fill_(-1.0)  # eager work between replays
        tv.project(G, x)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, g_eager), rep
        assert torch.equal(phi_g, phi_eager), rep
