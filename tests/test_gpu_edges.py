"""Edge cases of the binned likelihood on the GPU against the oracle: bin counts around
the 64-edge step (1, 63, 64, 65 bins) and on both sides of the LDS-table limit (500, 700),
two detectors, a single chain and a ragged batch,
for both waveforms, FP64 lnL and gradient and mixed lnL; and the autograd wrapper."""
import numpy as np
import pytest

from oracle import likelihood as L

from _events import near_draws, small_event
from gpu_common import WIDTHS, gpu_event, rb_condition_scale, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("approximant", ["taylorf2", "phenomd_nrtv2"])
# 500 bins with 3 detectors: the TaylorF2 FP64 gradient stages the edge tables in LDS
# (512 padded edges); 700 bins: too large for LDS, the global-table kernel.
@pytest.mark.parametrize("n_bins,n_det,B", [(1, 1, 1), (63, 2, 5), (64, 3, 64), (65, 2, 257), (500, 3, 9), (700, 3, 17)])
def test_edge_shapes(approximant, n_bins, n_det, B):
    ev = small_event(approximant=approximant, n_det=n_det, duration=4.0, f_high=512.0, n_bins=n_bins)
    L.prepare(ev)
    gev = gpu_event(ev)
    th = near_draws(ev.theta_ref, B, 70 + n_bins, scale=0.5)
    t = _cuda(th)
    want = L.loglike_rb(ev, th)
    scale = np.maximum(np.abs(want), rb_condition_scale(ev, th))
    got = gev.loglike(t).cpu().numpy()
    assert np.all(np.abs(got - want) <= 1e-8 * scale), np.abs(got - want).max()
    lg, g = gev.loglike_grad(t)
    lg, g = lg.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.abs(lg - want) <= 1e-8 * scale)
    wl, wg = L.loglike_rb_grad(ev, th)
    gs, ws = g * WIDTHS, wg * WIDTHS
    rel = np.abs(gs - ws).max(axis=1) / np.maximum(np.abs(ws).max(axis=1), 1e-300)
    say(approximant, n_bins, n_det, B, "lnL scaled err", (np.abs(got - want) / scale).max(), "grad", rel.max())
    assert np.all(rel <= 1e-5)
    gm = gev.loglike(t, precision="mixed").cpu().numpy()
    assert np.all(np.abs(gm - want) <= 1e-2)


def test_autograd_wrapper_returns_library_gradient():
    from paper_2404_11397_amd import LogLikeFn
    ev = small_event(duration=4.0, f_high=256.0, n_bins=40)
    L.prepare(ev)
    gev = gpu_event(ev)
    th = _cuda(near_draws(ev.theta_ref, 9, 80)).requires_grad_(True)
    w = _cuda(np.linspace(0.5, 1.5, 9))
    lnl = LogLikeFn.apply(th, gev)
    (lnl * w).sum().backward()
    _, g = gev.loglike_grad(th.detach())
    assert torch.equal(th.grad, w[:, None] * g)
