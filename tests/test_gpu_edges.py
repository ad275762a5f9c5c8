"""Edge cases of the binned likelihood on the GPU against the oracle: bin counts around
the 64-edge step (1, 63, 64, 65 bins) and on both sides of the LDS-table limits (500, 700
for TaylorF2; 1100 for IMRPhenomD_NRTidalv2), two detectors, a single chain and a ragged batch,
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
# (512 padded edges); 700 bins: too large for LDS, the global-table kernel.  The
# IMRPhenomD_NRTidalv2 FP64 gradient stages its tables up to 1024 padded edges at 3
# detectors; 1100 bins take its global-table kernel.  511 / 703 / 1023 bins with 3 / 2 / 1
# detectors are the largest TaylorF2 tables staged in LDS for each detector count (512, 704
# and 1024 padded edges: full and partial staging rounds per thread), 1024 bins with one
# detector the first that is not; the ragged batches leave the last 8-chain workgroup part
# empty.
@pytest.mark.parametrize("n_bins,n_det,B", [(1, 1, 1), (63, 2, 5), (64, 3, 64), (65, 2, 257), (500, 3, 9), (700, 3, 17),
                                            (1100, 3, 5), (511, 3, 13), (703, 2, 13), (1023, 1, 13), (1024, 1, 3)])
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


@pytest.mark.parametrize("approximant", ["taylorf2", "phenomd_nrtv2"])
def test_near_null_response(approximant):
    """Chains for which the first detector's response C_0 nearly vanishes (edge-on, iota =
    pi/2, and psi on the zero of F+): |K_0| ~ 1e-17, where the phase of K_0 is set by
    rounding.  lnL and gradient must still match the oracle."""
    from oracle import detector as Det
    ev = small_event(approximant=approximant, n_det=3, duration=4.0, f_high=512.0, n_bins=40)
    L.prepare(ev)
    gev = gpu_event(ev)
    th = near_draws(ev.theta_ref, 8, 91, scale=0.5)
    for i in range(0, 8, 2):
        ra, dec = th[i, 11], th[i, 12]
        a, _ = Det.antenna_patterns(ev.tensors[0], ra, dec, 0.0, ev.gmst)
        b, _ = Det.antenna_patterns(ev.tensors[0], ra, dec, np.pi / 4, ev.gmst)
        th[i, 9] = np.pi / 2
        th[i, 10] = 0.5 * np.arctan2(-a, b) % np.pi  # F+ of detector 0 vanishes
    c0 = [abs(W_proj) for W_proj in _response0(ev, th)]
    assert max(c0[0::2]) < 1e-14 and min(c0[1::2]) > 1e-3
    t = _cuda(th)
    want, wg = L.loglike_rb_grad(ev, th)
    scale = np.maximum(np.abs(want), rb_condition_scale(ev, th))
    lg, g = gev.loglike_grad(t)
    lg, g = lg.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.abs(lg - want) <= 1e-8 * scale)
    assert np.all(np.abs(gev.loglike(t).cpu().numpy() - want) <= 1e-8 * scale)
    gs, ws = g * WIDTHS, wg * WIDTHS
    rel = np.abs(gs - ws).max(axis=1) / np.maximum(np.abs(ws).max(axis=1), 1e-300)
    say(approximant, "near-null |C_0|", max(c0[0::2]), "grad", rel.max())
    assert np.all(rel <= 1e-5)
    gm = gev.loglike(t, precision="mixed").cpu().numpy()
    lm, _ = gev.loglike_grad(t, precision="mixed")
    assert np.all(np.abs(gm - want) <= 1e-2) and np.all(np.abs(lm.cpu().numpy() - want) <= 1e-2)


def _response0(ev, th):
    from oracle import waveform as W
    out = []
    for row in th:
        (c0, _), *_ = W.projection(W.unpack(row[None, :]), ev.tensors, ev.vertices, ev.gmst)
        out.append(complex(np.asarray(c0).ravel()[0]))
    return out


def test_random_event_sweep():
    """Seeded random small events (waveform, 1-3 detectors, 2-8 s, 256-1024 Hz, 5-1100 bins,
    1-69 chains, draws at three spreads): FP64 lnL of both kernels, the gradient and the mixed
    lnL against the oracle."""
    rng = np.random.default_rng(20261203)
    for case in range(12):
        ap = ["taylorf2", "phenomd_nrtv2"][case % 2]
        nd = int(rng.integers(1, 4))
        dur = float(rng.choice([2.0, 4.0, 8.0]))
        fh = float(rng.choice([256.0, 512.0, 1024.0]))
        npts = int((fh - 20.0) * dur) + 1
        nb = int(min(npts - 1, rng.choice([5, 37, 100, 300, 511, 600, 900, 1100])))
        B = int(rng.integers(1, 70))
        say("sweep case", case, ap, nd, dur, fh, nb, B)
        ev = small_event(approximant=ap, n_det=nd, duration=dur, f_high=fh, n_bins=nb, seed=case + 3)
        L.prepare(ev)
        gev = gpu_event(ev)
        th = near_draws(ev.theta_ref, B, 500 + case, scale=float(rng.choice([0.3, 1.0, 3.0])))
        t = _cuda(th)
        want, wg = L.loglike_rb_grad(ev, th)
        scale = np.maximum(np.abs(want), rb_condition_scale(ev, th))
        got = gev.loglike(t).cpu().numpy()
        lg, g = gev.loglike_grad(t)
        lg, g = lg.cpu().numpy(), g.cpu().numpy()
        assert np.all(np.abs(got - want) <= 1e-8 * scale)
        assert np.all(np.abs(lg - want) <= 1e-8 * scale)
        gs, ws = g * WIDTHS, wg * WIDTHS
        rel = np.abs(gs - ws).max(axis=1) / np.maximum(np.abs(ws).max(axis=1), 1e-300)
        assert np.all(rel <= 1e-5)
        assert np.all(np.abs(gev.loglike(t, precision="mixed").cpu().numpy() - want) <= 1e-2)
