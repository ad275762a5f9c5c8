"""rbl_loglike_grad_noalloc (no workspace, no allocation) called through the C-ABI gives the
results of rbl_loglike_grad, on two calls in a row (the second with a smaller batch, so
the static scratch still holds the first call's larger contents), for both waveforms and
both precisions; batches beyond the scratch are refused."""
import ctypes

import numpy as np
import pytest

from gpu_common import WIDTHS, gpu_event, oracle_event, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _noalloc(gev, theta, precision):
    from paper_2404_11397_amd import _lib
    from paper_2404_11397_amd.rbl import PRECISIONS
    B = theta.shape[0]
    lnl = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
    grad = torch.full((B, 13), np.nan, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().rbl_loglike_grad_noalloc(gev._h, ctypes.c_void_p(theta.data_ptr()), B,
                                                  PRECISIONS[precision], ctypes.c_void_p(lnl.data_ptr()),
                                                  ctypes.c_void_p(grad.data_ptr()), stream))
    return lnl, grad


def _check_same(got, want, precision):
    gl, gg = (x.cpu().numpy() for x in got)
    wl, wg = (x.cpu().numpy() for x in want)
    if precision == "fp64":
        scale = np.maximum(np.abs(wl), 1.0)
        assert np.max(np.abs(gl - wl) / scale) <= 1e-8
        gs, ws = gg * WIDTHS, wg * WIDTHS
        assert np.max(np.abs(gs - ws).max(axis=1) / np.maximum(np.abs(ws).max(axis=1), 1e-300)) <= 1e-5
    else:
        assert np.max(np.abs(gl - wl)) <= 1e-2
    # the same kernels on the same inputs: bitwise the same in practice
    say("  bitwise equal:", bool(np.array_equal(gl, wl) and np.array_equal(gg, wg)))


@pytest.mark.parametrize("name,big,small", [("tf2_1det_32s", 256, 37), ("nrtv2_3det_256s", 700, 65)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_workspace_entry_point(name, big, small, precision):
    say(f"noalloc {name} {precision} B={big} then B={small}")
    ev, w = oracle_event(name, batch=big, duration=8.0 if name.startswith("nrtv2") else None,
                         n_bins=200 if name.startswith("nrtv2") else None)
    gev = gpu_event(ev)
    th = torch.as_tensor(w["theta"], dtype=torch.float64, device="cuda")
    for B in (big, small):
        t = th[:B].contiguous()
        got = _noalloc(gev, t, precision)
        want = gev.loglike_grad(t, precision)
        torch.cuda.synchronize()
        _check_same(got, want, precision)


def test_noalloc_refuses_batches_beyond_the_scratch():
    from paper_2404_11397_amd import RblError, _lib
    ev, w = oracle_event("tf2_1det_32s", batch=8)
    gev = gpu_event(ev)
    B = _lib.RBL_NOALLOC_MAX_CHAINS + 1
    th = torch.zeros((B, 13), dtype=torch.float64, device="cuda")
    with pytest.raises(RblError) as ei:
        _noalloc(gev, th, "fp64")
    assert ei.value.code == -1
