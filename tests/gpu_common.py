"""Shared set-up of the GPU parity tests: the same seeded inputs go to the
oracle and to the library; the injection in the data is made by the oracle."""
import sys

import numpy as np

import synth
from oracle import binning
from oracle import likelihood as L
from oracle import waveform as W

# Prior widths of the GW170817 column (used to scale gradient components).
WIDTHS = np.array([0.03, 0.875, 0.1, 0.1, 5000.0, 5000.0, 74.0, 0.2, 2 * np.pi, np.pi, np.pi, 2 * np.pi, np.pi])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_event(name, batch=None, duration=None, n_bins=None, keep_b2=False):
    """Materialise a workload with an oracle injection; returns (oracle Event, workload dict)."""
    w = synth.workload(name, batch=batch, duration=duration, n_bins=n_bins)
    ev = L.Event(f=w["f"], delta_f=w["delta_f"], psd=w["psd"], data=None, tensors=w["tensors"],
                 vertices=w["vertices"], gmst=w["gmst"], approximant=w["waveform"], keep_b2=keep_b2)
    th0 = w["theta_inj"].copy()
    if np.isnan(th0[6]):
        th0[6] = 1.0
        snr1 = np.sqrt(L.optimal_snr2(ev, th0)[0])
        th0[6] = snr1 / w["snr"]
    h = W.strain(ev.f, th0, ev.tensors, ev.vertices, ev.gmst, ev.approximant, True)
    ev.data = np.stack([x[0] for x in h]) + w["noise"]
    ev.theta_ref = th0
    ev.edges = binning.pn_bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"])
    L.prepare(ev)
    w["theta_inj"] = th0
    return ev, w


def gpu_event(ev, keep_grid=False, device="cuda"):
    from paper_2404_11397_amd import Event
    return Event(ev.data, ev.psd, ev.tensors, ev.vertices, ev.gmst, ev.f[0], ev.delta_f, ev.theta_ref,
                 ev.edges, waveform=ev.approximant, keep_b2=ev.keep_b2, ref_taper=ev.ref_taper,
                 keep_grid=keep_grid, centre_nodes=ev.centre, device=device)


def rb_condition_scale(ev, theta):
    """Sum over detectors and bins of the magnitudes of the terms of the binned
    lnL (the reading of '1e-8 relative' used for values near zero)."""
    s = ev.summary
    fn = ev.f[ev.edges]
    tot = 0.0
    rc = L.node_ratios(ev, theta, L.bin_centres(ev)) if ev.centre else None
    for d, r in enumerate(L.node_ratios(ev, theta)):
        r0 = rc[d] if ev.centre else 0.5 * (r[:, 1:] + r[:, :-1])
        r1 = (r[:, 1:] - r[:, :-1]) / (fn[1:] - fn[:-1])
        tot = tot + (np.abs(s["A0"][d]) * np.abs(r0) + np.abs(s["A1"][d]) * np.abs(r1)
                     + 0.5 * s["B0"][d] * np.abs(r0) ** 2 + np.abs(s["B1"][d]) * np.abs(r0) * np.abs(r1)).sum(-1)
    return tot


def serving_oracle_event(eid):
    """Serving event `eid` with its configured injection, made by the oracle.  An
    IMRPhenomD_NRTidalv2 event whose untapered reference amplitude reaches zero inside the
    band (the ratio of Eq. (4) would be undefined there) is analysed on a band that ends at
    the last grid point where the tapered injection is non-zero, i.e. just below the end
    of the reference's taper.  Returns (oracle Event, spec, theta pool, band cut [Hz] or
    None)."""
    from oracle import phenomd_nrtv2
    sp = synth.serving_event(eid)
    x = synth.serving_inputs(sp)
    f_low, df, n = x["f_low"], x["delta_f"], x["n_freq"]
    f = f_low + df * np.arange(n)
    th0 = sp["theta_inj"]
    h = np.stack([y[0] for y in W.strain(f, th0, x["tensors"], x["vertices"], sp["gmst"], sp["waveform"], True)])
    cut = None
    if sp["waveform"] == "phenomd_nrtv2":
        a0 = np.ravel(phenomd_nrtv2.amplitude_factor(f, *th0[:6], taper=False))
        if np.any(a0 <= 0.0):
            n = int(np.nonzero(np.any(np.abs(h) > 0.0, axis=0))[0][-1]) + 1
            cut = float(f[n - 1])
    ev = L.Event(f=f[:n], delta_f=df, psd=x["psd"][:, :n], data=h[:, :n] + x["noise"][:, :n],
                 tensors=x["tensors"], vertices=x["vertices"], gmst=sp["gmst"], approximant=sp["waveform"])
    ev.theta_ref = th0
    ev.edges = binning.pn_bin_edges(f_low, df, n, sp["n_bins"])
    L.prepare(ev)
    return ev, sp, x["pool"], cut
