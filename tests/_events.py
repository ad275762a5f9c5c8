"""Small oracle events for the CPU pin tests (inputs from synth, waveform and
likelihood from the oracle)."""
import numpy as np

import synth
from oracle import binning
from oracle import likelihood as L
from oracle import waveform as W


def small_event(approximant="taylorf2", n_det=3, duration=4.0, f_high=512.0, n_bins=40,
                noise=True, snr=None, dl=60.0, keep_b2=False, ref_taper=False, seed=7):
    f_low, delta_f, n_freq, f = synth.frequency_grid(20.0, f_high, duration)
    psd = np.tile(synth.analytic_psd(f), (n_det, 1))
    sites = [(0.3, -1.2, 0.4), (-0.5, 2.0, 0.4), (0.9, 0.1, 1.3)][:n_det]
    geo = [synth.detector_geometry(*s) for s in sites]
    tensors = np.stack([g[0] for g in geo])
    vertices = np.stack([g[1] for g in geo])
    th0 = np.array([1.2, 0.8, 0.02, -0.01, 400.0, 700.0, dl, 0.01, 0.7, 0.9, 0.4, 2.1, -0.3])
    gmst = 0.37
    ev = L.Event(f=f, delta_f=delta_f, psd=psd, data=np.zeros_like(psd, complex),
                 tensors=tensors, vertices=vertices, gmst=gmst, approximant=approximant,
                 keep_b2=keep_b2, ref_taper=ref_taper)
    if snr is not None:
        th0[6] = th0[6] * np.sqrt(L.optimal_snr2(ev, th0)[0]) / snr
    h = W.strain(f, th0, tensors, vertices, gmst, approximant, True)
    data = np.stack([x[0] for x in h])
    if noise:
        data = data + synth.gaussian_noise(seed, psd, duration)
    ev.data = data
    ev.theta_ref = th0
    ev.edges = binning.pn_bin_edges(f_low, delta_f, n_freq, n_bins)
    return ev


def near_draws(theta0, n, seed, scale=1.0):
    """Parameter draws in a small box around theta0."""
    rng = np.random.default_rng(seed)
    width = np.array([2e-4, 0.05, 0.01, 0.01, 100.0, 100.0, 5.0, 2e-4, 0.2, 0.1, 0.1, 0.05, 0.05])
    th = theta0 + scale * width * rng.uniform(-1, 1, (n, 13))
    th[:, 9] = np.clip(th[:, 9], 0.01, np.pi - 0.01)
    return th
