"""tvreg_tv_grad_noalloc (no workspace, static device scratch) against
tvreg_tv_grad, the entry point it is a variant of: same kernels, so the
gradient and the TV value must agree bit for bit.  Two calls in a row, the
second on a smaller volume, so stale partial sums left in the shared scratch
by the first call cannot leak into the second."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tv():
    import paper_1105_4002_amd as tv
    return tv


def _volume(shape, seed, dtype):
    x = synth.random_volume(shape, seed, 0.0, 1.0)
    return torch.from_numpy(x).to(device="cuda:0", dtype=dtype)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_tv_grad_on_two_calls(tv, dtype):
    shapes = [(70, 80, 96), (5, 9, 17)]  # (nz, ny, nx): ragged, then smaller
    for i, shape in enumerate(shapes):
        print(f"noalloc call {i}: shape {shape} {dtype}", flush=True)
        x = _volume(shape, 40 + i, dtype)
        g_ref, v_ref = tv.tv_grad(x, 1e-4)
        out = torch.empty_like(x)
        val = torch.empty((), dtype=torch.float64, device=x.device)
        g, v = tv.tv_grad_noalloc(x, 1e-4, out=out, value_out=val)
        torch.cuda.synchronize()
        assert g.data_ptr() == out.data_ptr() and v.data_ptr() == val.data_ptr()
        assert torch.equal(g, g_ref)
        assert float(v.item()) == float(v_ref.item())
        if dtype == torch.float64 and i == 1:
            T_ref, grad_ref = oracle.tv(x.cpu().numpy(), 1e-4)
            assert abs(float(v.item()) - T_ref) <= 1e-12 * T_ref
            assert np.max(np.abs(g.cpu().numpy() - grad_ref)) <= 1e-12 * np.max(np.abs(grad_ref))


def test_noalloc_gradient_only_and_value_only(tv):
    x = _volume((16, 20, 24), 7, torch.float32)
    g_ref, v_ref = tv.tv_grad(x, 1e-4)
    g, v = tv.tv_grad_noalloc(x, 1e-4, value=False)
    assert v is None and torch.equal(g, g_ref)
    g, v = tv.tv_grad_noalloc(x, 1e-4, grad=False)
    torch.cuda.synchronize()
    assert g is None and float(v.item()) == float(v_ref.item())


def test_noalloc_rejects_volume_beyond_scratch(tv):
    x = torch.zeros(8, device="cuda:0")
    L = tv.lib()
    # 513^3 needs 9 x 129 x 33 TV blocks, more than the scratch holds; the
    # check precedes any device work, so nothing is read through x
    st = L.tvreg_tv_grad_noalloc(513, 513, 513, tv.F32, 1e-4, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(x.data_ptr()), None, None)
    assert st == tv.EINVAL
    assert b"at most 32768" in L.tvreg_last_error()
    # 512^3 is the largest cube it takes: validated, then rejected for the
    # missing outputs before any launch
    assert L.tvreg_tv_grad_noalloc(512, 512, 512, tv.F32, 1e-4, ctypes.c_void_p(x.data_ptr()),
                                   None, None, None) == tv.EINVAL
    assert b"neither gradient nor value" in L.tvreg_last_error()
