"""Reference-parameter search (Sec. II C) through the C-ABI: rbl_ref_search (a multistart of
CMA-ES runs on the device full-band lnL) follows the oracle's search generation by generation
when both get the same starts and normals (fitness from the GPU and from the oracle differ
only by rounding, so the rankings agree), and on a noise-free injection into the 3-detector
128 s TaylorF2 workload, from starting points drawn uniformly over the GW170817 prior box, it
finds the maximum: lnL(theta_inj) - lnL(best) below 13/2, the typical spread of lnL over a
13-parameter posterior, with the found point's lnL equal to the oracle's there."""
import numpy as np
import pytest

import synth
from gpu_common import gpu_event, say
from oracle import binning, cmaes
from oracle import likelihood as L
from oracle import waveform as W

from _events import small_event

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_ref_search_follows_the_oracle_cmaes():
    from paper_2404_11397_amd import ref_search
    ev = small_event(approximant="taylorf2", n_det=2, duration=8.0, f_high=512.0, n_bins=40)
    L.prepare(ev)
    gev = gpu_event(ev, keep_grid=True)
    half = np.array([1e-3, 0.1, 0.02, 0.02, 200, 200, 10, 1e-3, 0.5, 0.2, 0.2, 0.1, 0.1])
    lo, hi = ev.theta_ref - half, ev.theta_ref + half
    starts = np.stack([ev.theta_ref + 0.3 * half * np.sin(np.arange(13)),
                       ev.theta_ref - 0.5 * half * np.cos(np.arange(13))])
    normals = np.random.default_rng(8).standard_normal((2, 15, 16, 13))
    best, best_l, traces = ref_search(gev, lo, hi, starts, 0.2, normals)
    ob, obl, otraces = cmaes.search(lambda th: L.loglike_full(ev, th), lo, hi, starts, 0.2, 16, normals)
    for r in range(2):
        trace, otrace = traces[r], otraces[r]
        assert trace.shape == otrace.shape
        scale = np.abs(otrace[:, 0]).max()
        say(f"ref search vs oracle, run {r}: best lnL {trace[-1, 0]:.6f} / {otrace[-1, 0]:.6f}; max mean diff "
            f"(box units) {np.max(np.abs(trace[:, 2:] - otrace[:, 2:]) / (hi - lo)):.2e}")
        np.testing.assert_allclose(trace[:, 0], otrace[:, 0], rtol=0, atol=1e-9 * scale)
        np.testing.assert_allclose(trace[:, 1], otrace[:, 1], rtol=1e-9)
        assert np.max(np.abs(trace[:, 2:] - otrace[:, 2:]) / (hi - lo)) < 1e-9
    assert abs(best_l - obl) <= 1e-9 * abs(obl)
    np.testing.assert_allclose(best, ob, rtol=0, atol=1e-9 * np.max(hi - lo))


def test_ref_search_finds_a_noise_free_injection():
    from paper_2404_11397_amd import ref_search
    w = synth.workload("tf2_3det_128s", batch=1)
    th0 = w["theta_inj"]
    ev = L.Event(f=w["f"], delta_f=w["delta_f"], psd=w["psd"], data=None, tensors=w["tensors"],
                 vertices=w["vertices"], gmst=w["gmst"], approximant="taylorf2")
    ev.data = np.stack([x[0] for x in W.strain(w["f"], th0, w["tensors"], w["vertices"], w["gmst"], "taylorf2")])
    ev.theta_ref = th0
    ev.edges = binning.pn_bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"])
    gev = gpu_event(ev, keep_grid=True)
    b = synth.PRIORS["gw170817"]
    lo = np.array([b["Mc"][0], b["q"][0], b["chi"][0], b["chi"][0], b["L"][0], b["L"][0], b["dL"][0], b["tc"][0],
                   0.0, 0.0, 0.0, 0.0, -np.pi / 2])
    hi = np.array([b["Mc"][1], b["q"][1], b["chi"][1], b["chi"][1], b["L"][1], b["L"][1], b["dL"][1], b["tc"][1],
                   2 * np.pi, np.pi, np.pi, 2 * np.pi, np.pi / 2])
    rng = np.random.default_rng(21)
    starts = lo + rng.random((16, 13)) * (hi - lo)
    normals = rng.standard_normal((16, 400, 128, 13))
    best, best_l, traces = ref_search(gev, lo, hi, starts, 0.3, normals)
    peak = float(gev.loglike_full(torch.as_tensor(th0[None, :], device="cuda"))[0])
    want = L.loglike_full(ev, best[None, :])[0]
    finals = np.array([t[-1, 0] for t in traces])
    say(f"ref search, noise-free TaylorF2 injection: lnL peak {peak:.3f}, found {best_l:.3f} "
        f"(oracle {want:.3f}); Mc {best[0]:.7f} vs {th0[0]:.7f}, tc {best[7]:.6f} vs {th0[7]:.6f}; "
        f"runs within 13/2 of the peak: {int(np.sum(peak - finals <= 6.5))} of 16")
    assert abs(best_l - want) <= 1e-8 * max(abs(want), peak)
    assert peak - best_l <= 6.5


def test_ref_search_argument_checks():
    """Refused before any device work: a population below 4, no start, a start outside the
    box, an empty box, a non-positive step, and an event built without the full grid."""
    from paper_2404_11397_amd import RblError, ref_search
    ev = small_event(approximant="taylorf2", n_det=1, duration=4.0, f_high=256.0, n_bins=20)
    L.prepare(ev)
    gev = gpu_event(ev, keep_grid=True)
    lo, hi = ev.theta_ref - 0.1 * np.abs(ev.theta_ref) - 1e-3, ev.theta_ref + 0.1 * np.abs(ev.theta_ref) + 1e-3
    z = np.zeros((1, 2, 8, 13))
    cases = [
        (lo, hi, ev.theta_ref, 0.2, np.zeros((1, 2, 3, 13))),   # lambda < 4
        (lo, hi, hi + 1.0, 0.2, z),                               # start outside the box
        (hi, lo, ev.theta_ref, 0.2, z),                           # lo > hi
        (lo, hi, ev.theta_ref, 0.0, z),                           # sigma0 = 0
    ]
    for a, b, st, sig, nz in cases:
        with pytest.raises(RblError) as ei:
            ref_search(gev, a, b, st, sig, nz)
        assert ei.value.code == -1
    with pytest.raises(ValueError):
        ref_search(gev, lo, hi, ev.theta_ref, 0.2, np.zeros((2, 2, 8, 13)))  # one start, two sets of normals
    nogrid = gpu_event(ev, keep_grid=False)
    with pytest.raises(RblError) as ei:
        ref_search(nogrid, lo, hi, ev.theta_ref, 0.2, z)
    assert ei.value.code == -7
