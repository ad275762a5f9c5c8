"""Bin edges from a post-Newtonian phase-bound ansatz (Sec. II C).

The paper places bins so that the phase difference across a bin stays below
a threshold, using a PN ansatz for the phase that is independent of the source
parameters.  Reading used here: the ansatz phase
    Phi(f) = sum_g sgn(g) (f / f*_g)^g,  g in {-5/3, -2/3, 1, 5/3, 7/3},
    f*_g = f_low for g < 0 and f_high for g > 0,
is split into n_bins equal steps between the band ends; each step boundary is
snapped to the grid index whose Phi is nearest, and the indices are then made
strictly increasing with the first at 0 and the last at N - 1.  The bin count
replaces the threshold epsilon.  Edges are an input of the likelihood, so this
choice affects the accuracy of the binned likelihood, never its parity.
"""
import numpy as np

GAMMAS = (-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0)


def ansatz_phase(f, f_low, f_high):
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    for g in GAMMAS:
        fs = f_low if g < 0 else f_high
        out += np.sign(g) * (f / fs) ** g
    return out


def pn_bin_edges(f_low, delta_f, n_freq, n_bins):
    """Grid indices [n_bins + 1] of the bin edges (see module docstring)."""
    if n_bins < 1 or n_bins > n_freq - 1:
        raise ValueError("need 1 <= n_bins <= n_freq - 1")
    k = np.arange(n_freq)
    f = f_low + delta_f * k
    f_high = f[-1]
    phi = ansatz_phase(f, f_low, f_high)
    targets = phi[0] + (phi[-1] - phi[0]) * np.arange(n_bins + 1) / n_bins
    pos = np.searchsorted(phi, targets)              # first index with phi >= target
    pos = np.clip(pos, 1, n_freq - 1)
    below = phi[pos - 1]
    above = phi[pos]
    edges = np.where(targets - below <= above - targets, pos - 1, pos)
    edges[0] = 0
    edges[-1] = n_freq - 1
    for i in range(1, n_bins + 1):                    # strictly increasing
        edges[i] = max(edges[i], edges[i - 1] + 1)
    edges[-1] = n_freq - 1
    for i in range(n_bins - 1, -1, -1):
        edges[i] = min(edges[i], edges[i + 1] - 1)
    return edges.astype(np.int64)
