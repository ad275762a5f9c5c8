"""The workloads: shapes, seeds and injections (inputs only).

  tf2_1det_32s            TaylorF2, 1 detector, 32 s, 20-1024 Hz, 100 bins, 256 chains, SNR 30
  tf2_3det_128s           TaylorF2, 3 detectors, 128 s, 20-2048 Hz, 500 bins, 4096 chains
  nrtv2_3det_256s         IMRPhenomD_NRTidalv2, 3 detectors, 256 s, 20-2048 Hz, 1000 bins,
                          16384 chains, SNR 12
  *_grad8192              the same data, 8192 chains (lnL and gradient)
  serving                 64 events and a Poisson request stream (serving_event, serving_stream)

Seeds (PCG64): noise 1001 / 1002 / 1003, geometry and angles 2001 / 2002 / 2003, parameter
draws 3001 / 3002 / 3003 (3004 for the 8192-chain batches); serving events 5000 + event id,
serving arrivals 5999.

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


def _tf2_1det_32s():
    ang = _angles(2001)
    mc, q = component_to_chirp(1.5, 1.3)
    return dict(name="tf2_1det_32s", waveform="taylorf2", sites=[(0.0, 0.0, 0.0)], gmst=ang["gmst"],
                duration=32.0, f_low=20.0, f_high=1024.0, n_bins=100, batch=256,
                theta_inj=_theta(mc, q, 0.01, 0.01, 300.0, 500.0, None, 0.0, ang),
                snr=30.0, prior="injection", mc_window=None, seeds=(1001, 2001, 3001))


def _tf2_3det_128s():
    ang = _angles(2002)
    return dict(name="tf2_3det_128s", waveform="taylorf2", sites=_network3(2002), gmst=ang["gmst"],
                duration=128.0, f_low=20.0, f_high=2048.0, n_bins=500, batch=4096,
                theta_inj=_theta(1.1975, 0.85, 0.02, -0.01, 400.0, 600.0, 40.0, 0.0, ang),
                snr=None, prior="gw170817", mc_window=None, seeds=(1002, 2002, 3002))


def _nrtv2_3det_256s():
    ang = _angles(2003)
    mc, q = component_to_chirp(1.7, 1.6)
    # Same network as tf2_3det_128s ("same 3 detectors").
    return dict(name="nrtv2_3det_256s", waveform="phenomd_nrtv2", sites=_network3(2002), gmst=ang["gmst"],
                duration=256.0, f_low=20.0, f_high=2048.0, n_bins=1000, batch=16384,
                theta_inj=_theta(mc, q, 0.01, 0.01, 400.0, 400.0, None, 0.0, ang),
                snr=12.0, prior="gw190425", mc_window=(mc - 0.0025, mc + 0.0025),
                seeds=(1003, 2003, 3003))


CONFIGS = {"tf2_1det_32s": _tf2_1det_32s(), "tf2_3det_128s": _tf2_3det_128s(), "nrtv2_3det_256s": _nrtv2_3det_256s()}
# Differentiation workloads reuse the tf2_3det_128s / nrtv2_3det_256s data with 8192 chains.
CONFIGS["tf2_3det_128s_grad8192"] = dict(CONFIGS["tf2_3det_128s"], name="tf2_3det_128s_grad8192", batch=8192, seeds=(1002, 2002, 3004))
CONFIGS["nrtv2_3det_256s_grad8192"] = dict(CONFIGS["nrtv2_3det_256s"], name="nrtv2_3det_256s_grad8192", batch=8192, seeds=(1003, 2003, 3004))


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


# ---- serving workload: 64 resident events and a Poisson request stream ----------------------

N_SERVE_EVENTS = 64
SERVE_RATE_HZ = 200.0
SERVE_POOL = 2          # theta batches pre-drawn per event (requests cycle through them)


def serving_event(eid):
    """Event `eid` of the serving workload, everything from PCG64(5000 + eid):
    1-3 detectors at seeded sites, segment in {32, 64, 128, 256} s over 20-2048 Hz,
    100-1000 bins, TaylorF2 or IMRPhenomD_NRTidalv2 (even odds), 256-4096 chains,
    injection from the "injection" prior column; its requests draw theta from that
    column with the chirp mass narrowed to +-0.005 around the injection."""
    rng = np.random.Generator(np.random.PCG64(5000 + eid))
    n_det = int(rng.integers(1, 4))
    duration = float(rng.choice([32.0, 64.0, 128.0, 256.0]))
    n_bins = int(rng.integers(100, 1001))
    waveform = "taylorf2" if rng.uniform() < 0.5 else "phenomd_nrtv2"
    batch = int(rng.integers(256, 4097))
    sites = []
    for _ in range(n_det):
        sites.append((float(np.arcsin(rng.uniform(-0.9, 0.9))), float(rng.uniform(-np.pi, np.pi)),
                      float(rng.uniform(0, np.pi))))
    gmst = float(rng.uniform(0, 2 * np.pi))
    th = draw_theta(int(rng.integers(1 << 31)), 1, "injection")[0]
    win = (th[0] - 0.005, th[0] + 0.005)
    pool_seeds = [int(rng.integers(1 << 31)) for _ in range(SERVE_POOL)]
    return dict(eid=eid, n_det=n_det, duration=duration, n_bins=n_bins, waveform=waveform, batch=batch,
                sites=sites, gmst=gmst, theta_inj=th, mc_window=win, noise_seed=int(rng.integers(1 << 31)),
                pool_seeds=pool_seeds, f_low=20.0, f_high=2048.0)


def serving_inputs(spec):
    """Grid, PSD, geometry, noise and the theta pool of one serving event."""
    f_low, delta_f, n_freq, f = frequency_grid(spec["f_low"], spec["f_high"], spec["duration"])
    nd = spec["n_det"]
    psd = np.tile(analytic_psd(f), (nd, 1))
    geo = [detector_geometry(*s) for s in spec["sites"]]
    pool = [draw_theta(s, spec["batch"], "injection", spec["mc_window"]) for s in spec["pool_seeds"]]
    return dict(f_low=f_low, delta_f=delta_f, n_freq=n_freq, psd=psd,
                tensors=np.stack([g[0] for g in geo]), vertices=np.stack([g[1] for g in geo]),
                noise=gaussian_noise(spec["noise_seed"], psd, spec["duration"]), pool=pool)


def serving_stream(n_requests, rate_hz=SERVE_RATE_HZ, seed=5999, n_events=N_SERVE_EVENTS):
    """Request stream: arrival offsets [s] with Exp(rate) gaps, the event of each
    request (uniform over the events) and the pool index it uses."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    events = rng.integers(0, n_events, n_requests)
    pools = rng.integers(0, SERVE_POOL, n_requests)
    return np.cumsum(gaps), events, pools
