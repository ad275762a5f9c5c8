"""Whittle likelihood on the full grid and its relative-binned form.

Full grid (Sec. II A, Eqs. 2-3): with <a, b>_c = 4 df sum_k a_k conj(b_k) / S_k
over the grid f_k = f_low + k df (both band ends included) and
<a, b> = Re <a, b>_c,
    lnL(theta) = sum_d [ Re <d_d, h_d>_c - <h_d, h_d> / 2 ],
i.e. Eq. (2) with the theta-independent -<d, d>/2 dropped (the paper's
"+ constant"), so a noise-free injection peaks at <h, h>/2.

Relative binning (Sec. II C, Eqs. 4-5), step by step:
  1. bins: bin b holds grid indices e_b <= k < e_{b+1}; the last bin also holds
     k = e_{Nb} = N - 1; f_m(b) = (f_{e_b} + f_{e_{b+1}}) / 2 is its centre;
  2. h0_d = h_d(.; theta0), the reference waveform (for IMRPhenomD_NRTidalv2
     generated without the Planck taper unless requested, Sec. II C 1);
  3. summary data per (detector, bin), exact sums over the bin:
       A0 = 4 df sum d h0*/S,           A1 = 4 df sum d h0*/S (f - f_m),
       B0 = 4 df sum |h0|^2/S,          B1 = 4 df sum |h0|^2/S (f - f_m),
       B2 = 4 df sum |h0|^2/S (f - f_m)^2   (kept only on request);
  4. ratio at the bin edges r_j = h(f_j; theta) / h0(f_j)   (Eq. 4);
  5. linear model r = r0 + r1 (f - f_m) through the edge values   (Eq. 5):
       r0 = (r_b + r_{b+1}) / 2,  r1 = (r_{b+1} - r_b) / (f_{b+1} - f_b);
  6. substitute into the full-grid expression:
       lnL = sum_d sum_b [ Re(A0 r0* + A1 r1*) - B0 |r0|^2 / 2
                           - B1 Re(r0 r1*) - B2 |r1|^2 / 2 ].
Centre-node variant (Event.centre): Eq. (5) expands the ratio about the bin centre, so
r0 is taken as the ratio evaluated at f_m(b) itself, r0 = r(f_m), and r1 from the
edges as above: 2 Nb + 1 waveform evaluations per chain instead of Nb + 1.  The summary
data are the same; the B2 term is not offered with this variant.
"""
from dataclasses import dataclass, field

import numpy as np

from . import ad, waveform


@dataclass
class Event:
    f: np.ndarray                 # [N] grid
    delta_f: float
    psd: np.ndarray               # [D, N]
    data: np.ndarray              # [D, N] complex
    tensors: np.ndarray           # [D, 3, 3]
    vertices: np.ndarray          # [D, 3]
    gmst: float
    approximant: str
    edges: np.ndarray = None      # [Nb + 1] grid indices
    theta_ref: np.ndarray = None  # [13]
    keep_b2: bool = False
    ref_taper: bool = False       # taper the reference (the paper's runs do not)
    centre: bool = False          # r0 from the ratio at the bin centre (2 Nb + 1 evaluations)
    summary: dict = field(default=None, repr=False)


def inner_c(a, b, psd, delta_f):
    """<a, b>_c = 4 df sum a conj(b) / S along the last axis."""
    return 4.0 * delta_f * (a * np.conj(b) / psd).sum(axis=-1)


def loglike_full(ev, theta, taper=True):
    """Full-grid lnL for theta [B, 13] -> [B] (Dual if theta holds Duals)."""
    hs = waveform.strain(ev.f, theta, ev.tensors, ev.vertices, ev.gmst, ev.approximant, taper)
    total = 0.0
    for d, h in enumerate(hs):
        w = 4.0 * ev.delta_f / ev.psd[d]
        dh = (h.conj() * (ev.data[d] * w)).sum(axis=-1).real
        hh = ((h * h.conj()).real * w).sum(axis=-1)
        total = total + dh - 0.5 * hh
    return total


def optimal_snr2(ev, theta, taper=True):
    """Network <h, h> (the optimal SNR squared) for theta [B, 13] -> [B]."""
    hs = waveform.strain(ev.f, theta, ev.tensors, ev.vertices, ev.gmst, ev.approximant, taper)
    return sum((np.abs(h) ** 2 * 4.0 * ev.delta_f / ev.psd[d]).sum(axis=-1)
               for d, h in enumerate(hs))


def bin_index(n_freq, edges):
    """Bin of every grid point (last bin closed on the right)."""
    idx = np.searchsorted(np.asarray(edges), np.arange(n_freq), side="right") - 1
    return np.minimum(idx, len(edges) - 2)


def summary_data(ev):
    """Steps 1-3: A0, A1 (complex) and B0, B1, B2 (real), each [D, Nb]."""
    edges = np.asarray(ev.edges)
    nb = len(edges) - 1
    f = ev.f
    taper = ev.ref_taper
    h0 = waveform.strain(f, ev.theta_ref, ev.tensors, ev.vertices, ev.gmst, ev.approximant, taper)
    fe = f[edges]
    fm = 0.5 * (fe[:-1] + fe[1:])
    b_of_k = bin_index(len(f), edges)
    dfm = f - fm[b_of_k]
    out = {k: [] for k in ("A0", "A1", "B0", "B1", "B2")}
    for d in range(len(h0)):
        h = h0[d][0]
        w = 4.0 * ev.delta_f / ev.psd[d]
        dh = ev.data[d] * np.conj(h) * w
        hh = (np.abs(h) ** 2) * w
        a0 = np.zeros(nb, complex)
        a1 = np.zeros(nb, complex)
        b0 = np.zeros(nb)
        b1 = np.zeros(nb)
        b2 = np.zeros(nb)
        for b in range(nb):
            lo = edges[b]
            hi = edges[b + 1] + (1 if b == nb - 1 else 0)
            s = slice(lo, hi)
            a0[b] = dh[s].sum()
            a1[b] = (dh[s] * dfm[s]).sum()
            b0[b] = hh[s].sum()
            b1[b] = (hh[s] * dfm[s]).sum()
            b2[b] = (hh[s] * dfm[s] ** 2).sum()
        for k, v in zip(("A0", "A1", "B0", "B1", "B2"), (a0, a1, b0, b1, b2)):
            out[k].append(v)
    return {k: np.array(v) for k, v in out.items()}


def prepare(ev):
    """Compute and attach the summary data (the 'set_event' step)."""
    ev.summary = summary_data(ev)
    return ev


def bin_centres(ev):
    """f_m(b) = (f_{e_b} + f_{e_{b+1}}) / 2."""
    fe = ev.f[np.asarray(ev.edges)]
    return 0.5 * (fe[:-1] + fe[1:])


def node_ratios(ev, theta, freqs=None):
    """Step 4: r_d(f_j) = h_d(f_j; theta) / h0_d(f_j) at the bin edges (or at `freqs`)
    -> list over d of [B, len]."""
    fn = ev.f[np.asarray(ev.edges)] if freqs is None else freqs
    h = waveform.strain(fn, theta, ev.tensors, ev.vertices, ev.gmst, ev.approximant, True)
    h0 = waveform.strain(fn, ev.theta_ref, ev.tensors, ev.vertices, ev.gmst, ev.approximant,
                         ev.ref_taper)
    return [hd / h0d[0] for hd, h0d in zip(h, h0)]


def loglike_rb(ev, theta):
    """Steps 4-6: relative-binned lnL for theta [B, 13] -> [B]."""
    if ev.summary is None:
        prepare(ev)
    s = ev.summary
    fn = ev.f[np.asarray(ev.edges)]
    width = fn[1:] - fn[:-1]
    total = 0.0
    centre = node_ratios(ev, theta, bin_centres(ev)) if ev.centre else None
    for d, r in enumerate(node_ratios(ev, theta)):
        rl, rr = r[..., :-1], r[..., 1:]
        r0 = centre[d] if ev.centre else 0.5 * (rl + rr)
        r1 = (rr - rl) / width
        r0c, r1c = r0.conj(), r1.conj()
        t = (s["A0"][d] * r0c + s["A1"][d] * r1c).real \
            - 0.5 * s["B0"][d] * (r0 * r0c).real - s["B1"][d] * (r0 * r1c).real
        if ev.keep_b2:
            if ev.centre:
                raise ValueError("the B2 term is not offered with the centre-node variant")
            t = t - 0.5 * s["B2"][d] * (r1 * r1c).real
        total = total + t.sum(axis=-1)
    return total


def theta_duals(theta):
    """Seed the 13 parameters of theta [B, 13] as Duals with shape [B, 1]."""
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    out = []
    for i in range(13):
        d = np.zeros((13, theta.shape[0], 1))
        d[i] = 1.0
        out.append(ad.Dual(theta[:, i:i + 1], d))
    return out


def loglike_rb_grad(ev, theta):
    """(lnL [B], d lnL / d theta [B, 13]) by forward-mode dual numbers."""
    res = loglike_rb(ev, theta_duals(theta))
    return res.v, res.d.T


def loglike_full_grad(ev, theta, taper=True):
    res = loglike_full(ev, theta_duals(theta), taper)
    return res.v, res.d.T
