"""The allocation-free closure inference entry point against the workspace
one: olb_closure_forward_noalloc (parameters from device memory, scratch in
a static device array) must give what olb_closure_forward gives for the
same parameters, normalisation and projection, on two calls in a row, the
second on a smaller lattice (the scratch keeps the first call's contents).
"""
import ctypes

import numpy as np
import pytest

import olb_inputs as I

pytestmark = pytest.mark.gpu


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1702_01690_amd import olb
    return torch, olb


def _case(nx, ny, seed):
    params = I.closure_params(seed=seed, last_scale=1.0)
    m = I.closure_moments(nx, ny, seed=seed + 1)
    ref = m + 0.01 * (I.closure_moments(nx, ny, seed=seed + 2) - m)
    norm = (m.mean(axis=(1, 2)), m.std(axis=(1, 2)), np.abs(ref - m).std(axis=(1, 2)))
    return params, m, norm


def _with_workspace(torch, olb, nx, ny, params, m, norm, mask, stream):
    nbytes = olb.olb_closure_workspace_bytes(nx, ny)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    h = olb.olb_closure_init(nx, ny, ws.data_ptr(), nbytes, stream.cuda_stream)
    try:
        olb.olb_closure_set_norm(h, *norm)
        olb.olb_closure_set_params(h, params)
        olb.olb_closure_set_conserve(h, mask)
        dm = torch.tensor(m.ravel(), dtype=torch.float64, device="cuda:0")
        out = torch.empty_like(dm)
        olb.olb_closure_forward(h, dm.data_ptr(), out.data_ptr())
        stream.synchronize()
        return out.cpu().numpy().reshape(4, ny, nx)
    finally:
        olb.olb_closure_free(h)


def _without(torch, olb, nx, ny, params, m, norm, mask, stream):
    dp = torch.tensor(np.asarray(params, dtype=np.float32), device="cuda:0")
    dm = torch.tensor(m.ravel(), dtype=torch.float64, device="cuda:0")
    out = torch.full_like(dm, np.nan)
    olb.olb_closure_forward_noalloc(nx, ny, dp.data_ptr(), *norm, mask, dm.data_ptr(), out.data_ptr(),
                                    stream.cuda_stream)
    stream.synchronize()
    return out.cpu().numpy().reshape(4, ny, nx)


@pytest.mark.parametrize("mask", [0, 7])
def test_noalloc_forward_equals_workspace_forward_on_two_calls(mask):
    torch, olb = _env()
    stream = torch.cuda.Stream()
    # first a ragged lattice (tiles of 16 nodes), then a smaller one
    for nx, ny, seed in ((100, 75, 3), (37, 21, 5)):
        params, m, norm = _case(nx, ny, seed)
        print(f"[noalloc] {nx}x{ny} mask={mask}", flush=True)
        want = _with_workspace(torch, olb, nx, ny, params, m, norm, mask, stream)
        got = _without(torch, olb, nx, ny, params, m, norm, mask, stream)
        assert np.all(np.isfinite(got))
        # same kernels, same operands, channel sums added in a fixed order:
        # the same bits
        np.testing.assert_array_equal(got, want)


def test_noalloc_forward_rejects_bad_arguments():
    torch, olb = _env()
    params, m, norm = _case(8, 8, 3)
    dp = torch.tensor(np.asarray(params, dtype=np.float32), device="cuda:0")
    dm = torch.tensor(m.ravel(), dtype=torch.float64, device="cuda:0")
    out = torch.empty_like(dm)
    for nx, ny, mask, nrm in ((0, 8, 0, norm), (8, 8, 16, norm), (1 << 16, 1 << 14, 0, norm),
                              (8, 8, 0, (norm[0], -norm[1], norm[2]))):
        with pytest.raises(olb.OlbError) as e:
            olb.olb_closure_forward_noalloc(nx, ny, dp.data_ptr(), *nrm, mask, dm.data_ptr(), out.data_ptr(), 0)
        assert e.value.code == olb.OLB_E_ARG
    with pytest.raises(olb.OlbError):
        olb.olb_closure_forward_noalloc(8, 8, 0, *norm, 0, dm.data_ptr(), out.data_ptr(), 0)
