"""The five workloads: shapes, seeds and injections (inputs only).

Seeds: noise = 1000 + cfg, geometry/angles = 2000 + cfg, parameter draws =
3000 + cfg, serving events = 5000 + event id, serving arrivals = 5999.

Where a workload fixes the signal-to-noise ratio instead of the distance, the
injection's distance is left as None here; the caller scales it with its own
waveform code (the tests use the oracle, the benchmark the library).
"""
import numpy as np

from .inputs import (analytic_psd, component_to_chirp, detector_geometry,
                     draw_theta, frequency_grid, gaussian_noise)


def _angles(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return {"phic": rng.uniform(0, 2 * np.pi), "iota": np.arccos(rng.uniform(-1, 1)),
            "psi": rng.uniform(0, np.pi), "ra": rng.uniform(0, 2 * np.pi),
            "dec": np.arcsin(rng.uniform(-1, 1)), "gmst": rng.uniform(0, 2 * np.pi)}


def _network3(seed):
    """Two co-aligned interferometers (same local arm azimuth) plus a third at
    its own azimuth, all at seeded sites."""
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    beta = rng.uniform(0, np.pi)
    sites = []
    for k in range(3):
        lat = np.arcsin(rng.uniform(-0.9, 0.9))
        lon = rng.uniform(-np.pi, np.pi)
        az = beta if k < 2 else rng.uniform(0, np.pi)
        sites.append((lat, lon, az))
    return sites


def _theta(mc, q, chi1, chi2, l1, l2, dl, tc, ang):
    return np.array([mc, q, chi1, chi2, l1, l2, np.nan if dl is None else dl, tc,
                     ang["phic"], ang["iota"], ang["psi"], ang["ra"], ang["dec"]])


def _cfg1():
    ang = _angles(2001)
    mc, q = component_to_chirp(1.5, 1.3)
    return dict(name="cfg1", waveform="taylorf2", sites=[(0.0, 0.0, 0.0)], gmst=ang["gmst"],
                duration=32.0, f_low=20.0, f_high=1024.0, n_bins=100, batch=256,
                theta_inj=_theta(mc, q, 0.01, 0.01, 300.0, 500.0, None, 0.0, ang),
                snr=30.0, prior="injection", mc_window=None, seeds=(1001, 2001, 3001))


def _cfg2():
    ang = _angles(2002)
    return dict(name="cfg2", waveform="taylorf2", sites=_network3(2002), gmst=ang["gmst"],
                duration=128.0, f_low=20.0, f_high=2048.0, n_bins=500, batch=4096,
                theta_inj=_theta(1.1975, 0.85, 0.02, -0.01, 400.0, 600.0, 40.0, 0.0, ang),
                snr=None, prior="gw170817", mc_window=None, seeds=(1002, 2002, 3002))


def _cfg3():
    ang = _angles(2003)
    mc, q = component_to_chirp(1.7, 1.6)
    # Same network as cfg2 ("same 3 detectors").
    return dict(name="cfg3", waveform="phenomd_nrtv2", sites=_network3(2002), gmst=ang["gmst"],
                duration=256.0, f_low=20.0, f_high=2048.0, n_bins=1000, batch=16384,
                theta_inj=_theta(mc, q, 0.01, 0.01, 400.0, 400.0, None, 0.0, ang),
                snr=12.0, prior="gw190425", mc_window=(mc - 0.0025, mc + 0.0025),
                seeds=(1003, 2003, 3003))


CONFIGS = {"cfg1": _cfg1(), "cfg2": _cfg2(), "cfg3": _cfg3()}
# Differentiation workloads reuse the cfg2 / cfg3 data with 8192 chains.
CONFIGS["cfg4_tf2"] = dict(CONFIGS["cfg2"], name="cfg4_tf2", batch=8192, seeds=(1002, 2002, 3004))
CONFIGS["cfg4_nrtv2"] = dict(CONFIGS["cfg3"], name="cfg4_nrtv2", batch=8192, seeds=(1003, 2003, 3004))


def workload(name, batch=None, duration=None, n_bins=None):
    """Materialise a workload's inputs.

    Returns a dict with the grid, PSD [D, N], noise [D, N], detector tensors
    [D, 3, 3] and vertices [D, 3], gmst, the injection parameters (distance may
    be NaN when an SNR target is given), the parameter draws [B, 13] and the
    bin count.  `batch`, `duration` and `n_bins` shrink a workload for tests.
    """
    c = dict(CONFIGS[name])
    if duration is not None:
        c["duration"] = duration
    if n_bins is not None:
        c["n_bins"] = n_bins
    b = c["batch"] if batch is None else batch
    f_low, delta_f, n_freq, f = frequency_grid(c["f_low"], c["f_high"], c["duration"])
    nd = len(c["sites"])
    psd = np.tile(analytic_psd(f), (nd, 1))
    geo = [detector_geometry(*s) for s in c["sites"]]
    tensors = np.stack([g[0] for g in geo])
    vertices = np.stack([g[1] for g in geo])
    noise = gaussian_noise(c["seeds"][0], psd, c["duration"])
    theta = draw_theta(c["seeds"][2], b, c["prior"], c["mc_window"])
    return dict(name=c["name"], waveform=c["waveform"], f_low=f_low, delta_f=delta_f,
                n_freq=n_freq, f=f, psd=psd, noise=noise, tensors=tensors,
                vertices=vertices, gmst=c["gmst"], theta_inj=c["theta_inj"].copy(),
                snr=c["snr"], theta=theta, n_bins=c["n_bins"], duration=c["duration"])
