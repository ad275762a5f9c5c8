"""Benchmark: relative-binned lnL + gradient evaluations per second on one GPU.

Workload (the differentiation configuration on the 3-detector TaylorF2 data):
3 detectors, 128 s segment, 20-2048 Hz (259585 grid points per detector),
500 relative-binning bins, 8192 chains drawn from the GW170817 prior column,
lnL and the 13-parameter gradient in FP64 (the gradient-based local MCMC
step).  Synthetic data: the library's own TaylorF2 injection plus seeded
Gaussian noise from the analytic PSD; all inputs resident in HBM before the
timed region.  One step = one rbl_loglike_grad call over the batch (per-chain
setup kernel + fused adjoint kernel).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

# Peaks of one MI355X (vendor figures): FP64 vector 78.6 TFLOP/s, HBM 8 TB/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def flops_per_eval(n_nodes, n_det, grad, waveform="taylorf2"):
    """Algorithmic FP64 flops of one chain's relative-binned lnL (+ gradient), counted
    from the operations the method needs (FMA = 2, add/mul = 1, a division 10, an exp
    or log 20, each sin/cos pair of a phase in revolutions at its minimal polynomial
    cost: exact reduction 2 + 17 FMA = 36).

    Per edge and detector: phase with delay (2), sin/cos (36), ratio K u (6), the binned
    terms and their sums (14); the gradient adds the edge adjoint and its sums (26).
    Per edge, TaylorF2: phase in the separable basis (8 mul + 10 FMA = 28); gradient:
    basis accumulations (20).  IMRPhenomD_NRTidalv2: point-particle phase, NRTidal Pade
    phase and tidal amplitude with its power-law term (110) and the amplitude ratio
    (2 per detector); gradient: the node-parameter adjoint (180).  Per chain: setup 600
    (TaylorF2) / 1500 (NRTidalv2) for lnL, 6000 / 18000 with the Jacobian.
    """
    if waveform == "taylorf2":
        per_node = 28 + n_det * (2 + 36 + 6 + 14)
        setup = 600
        if grad:
            per_node += n_det * 26 + 20
            setup = 6000
    else:
        per_node = 110 + n_det * (2 + 36 + 2 + 6 + 14)
        setup = 1500
        if grad:
            per_node += n_det * 26 + 180
            setup = 18000
    return n_nodes * per_node, setup


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--no-nrtv2", action="store_true", help="skip the IMRPhenomD_NRTidalv2 forms")
    p.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    p.add_argument("--serve-requests", type=int, default=2000)
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a plain device copy of known size (HBM counter calibration)")
    return p.parse_args()


def build_event(torch, workload, keep_grid=False):
    import synth
    from paper_2404_11397_amd import Event, bin_edges, strain
    w = synth.workload(workload)
    dev = torch.device("cuda:0")
    edges = bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"])
    th0 = w["theta_inj"].copy()
    psd_d = torch.as_tensor(w["psd"], device=dev)
    if np.isnan(th0[6]):  # distance set by an SNR target: <h, h> scales as 1/dL^2
        th0[6] = 1.0
        h1 = strain(w["waveform"], w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"],
                    w["n_freq"], th0, device=dev)
        rho1 = float(torch.sqrt(4.0 * w["delta_f"] * (h1.abs() ** 2 / psd_d).sum()))
        th0[6] = rho1 / w["snr"]
        w["theta_inj"] = th0
    h = strain(w["waveform"], w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"],
               w["n_freq"], th0, device=dev)
    data = h + torch.as_tensor(w["noise"], device=dev)
    psd = torch.as_tensor(w["psd"], device=dev)
    ev = Event(data, psd, w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"], th0, edges,
               waveform=w["waveform"], keep_grid=keep_grid, device=dev)
    return ev, w, edges, data


def cpu_baseline(w, edges, data_host, theta, seconds):
    """Time the FP64 oracle (lnL + dual-number gradient) on a bounded sample."""
    from oracle import likelihood as L
    ev = L.Event(f=w["f"], delta_f=w["delta_f"], psd=w["psd"], data=data_host, tensors=w["tensors"],
                 vertices=w["vertices"], gmst=w["gmst"], approximant=w["waveform"],
                 edges=np.asarray(edges), theta_ref=w["theta_inj"])
    L.prepare(ev)
    chunk = 32
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        lo = done % len(theta)
        L.loglike_rb_grad(ev, theta[lo:lo + chunk])
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} chain evaluations cycling through the batch in chunks of {chunk} "
                      f"(lnL + dual-number gradient), {dt:.1f} s, numpy FP64 single thread"}


TIMING_EVERY = 8  # kernel start/stop events on the first and every 8th call of a timed region


def time_calls(torch, fn, steps, warmup):
    """Wall time per call and HIP-event kernel times (main, setup) per timed call.  The events
    are taken inside the timed region on a sample of the calls (TIMING_EVERY): each timed call
    costs a few microseconds of device time."""
    from paper_2404_11397_amd import profile_enable, profile_read
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    profile_enable(True, every=TIMING_EVERY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    main_ms, setup_ms, calls = profile_read()
    profile_enable(False)
    return elapsed, main_ms / calls * 1e3, setup_ms / calls * 1e3


def flops_full_point(n_det):
    """Algorithmic FP64 flops per grid point of the full-band TaylorF2 lnL (Eqs. (2)-(3)):
    x = f^(1/3) (20), 1/x (10), ln x (20), amplitude x^-3.5 (23), basis phase (28); per
    detector the phase with delay (2), sin/cos (36), the projected strain (8), 1/S (10) and
    the two inner-product terms (8)."""
    return 101 + n_det * 64


def full_band(torch, steps):
    """Full-band lnL (every grid point, no binning) on the 1-detector 32 s workload beside the
    binned FP64 lnL on the same batch: throughput, and the binning error of Eq. (5)."""
    ev, w, edges, data = build_event(torch, "tf2_1det_32s", keep_grid=True)
    th = torch.as_tensor(w["theta"], device="cuda:0")
    B = th.shape[0]
    ws = ev.workspace(B, False)
    full = torch.empty(B, dtype=torch.float64, device="cuda:0")
    rb = torch.empty_like(full)
    el_f, ku_f, su_f = time_calls(torch, lambda: ev.loglike_full(th, out=full, workspace=ws), steps, 3)
    el_b, ku_b, su_b = time_calls(torch, lambda: ev.loglike(th, out=rb, workspace=ws), steps, 3)
    torch.cuda.synchronize()
    err = (rb - full).abs()
    # The binning error where a sampler spends its time: draws around the injection with the
    # spread of a diagonal inverse-Fisher estimate (sigma_i = 1 / |d lnL / d theta_i| there).
    th0 = w["theta_inj"]
    rng = np.random.default_rng(91)
    probe = torch.as_tensor(th0 + 1e-9 * np.abs(th0) * rng.standard_normal((64, 13)), device="cuda:0")
    g = ev.loglike_grad(probe)[1].cpu().numpy()
    sigma = np.minimum(1.0 / np.sqrt(np.mean(g * g, axis=0) + 1e-300), 0.05 * np.abs(th0) + 1e-3)
    near = th0 + sigma * rng.standard_normal((B, 13))
    near[:, 1] = np.clip(near[:, 1], 0.05, 1.0)
    near[:, 2:4] = np.clip(near[:, 2:4], -0.99, 0.99)
    near[:, 4:6] = np.maximum(near[:, 4:6], 0.0)
    near[:, 9] = np.clip(near[:, 9], 1e-3, np.pi - 1e-3)
    near[:, 12] = np.clip(near[:, 12], -np.pi / 2 + 1e-3, np.pi / 2 - 1e-3)
    tn = torch.as_tensor(near, device="cuda:0")
    full_n = ev.loglike_full(tn)
    err_n = (ev.loglike(tn) - full_n).abs()
    fl = flops_full_point(len(w["tensors"])) * w["n_freq"] * B
    return {"workload": "TaylorF2 lnL, 1 det, 32 s, 20-1024 Hz (%d points), %d bins, %d chains" % (w["n_freq"], w["n_bins"], B),
            "full_evals_per_s": B * steps / el_f, "full_kernel_us": ku_f,
            "full_est_tflops": fl / (ku_f * 1e-6) / 1e12,
            "full_est_frac_fp64_peak": fl / (ku_f * 1e-6) / 1e12 / PEAK_FP64_TFLOPS,
            "binned_evals_per_s": B * steps / el_b, "binned_kernel_us": ku_b,
            "kernel_speedup": ku_f / ku_b,
            "binning_error_near_injection": {
                "max_abs": float(err_n.max()), "median_abs": float(err_n.median()),
                "lnl_range": [float(full_n.min()), float(full_n.max())],
                "what": "chains drawn around the injection with the inverse-Fisher diagonal spread"},
            "binning_error_prior_draws": {
                "max_abs": float(err.max()), "median_abs": float(err.median()),
                "what": "the workload's prior-wide draws, far from the reference, where the linear "
                        "model of Eq. (5) is not meant to hold"}}


def summary_pass(torch, w, edges, data, psd, repeats=3):
    """Average duration of the summary-data kernels of rbl_event_create (HIP events)."""
    from paper_2404_11397_amd import Event, profile_enable, profile_read_summary
    profile_enable(True)
    profile_read_summary()
    for _ in range(repeats):
        Event(data, psd, w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"], w["theta_inj"], edges,
              waveform=w["waveform"], device=data.device)
    ms, n = profile_read_summary()
    profile_enable(False)
    return ms / n * 1e3


COPY_BYTES = 256 << 20   # the calibration copy reads and writes this many bytes per launch


def calibrate_copy(torch, repeats=10):
    """Plain copies of COPY_BYTES between two device buffers, one kernel per launch: the
    runtime's copy (hipMemcpyAsync device to device) and an elementwise kernel (y = x + 0).
    The FETCH_SIZE / WRITE_SIZE counters of these launches give the scale from counter
    units to HBM bytes."""
    x = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(repeats):
        y.copy_(x)
    torch.cuda.synchronize()
    for _ in range(repeats):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    return {"bytes_read_per_launch": COPY_BYTES, "bytes_written_per_launch": COPY_BYTES, "launches": repeats,
            "kernels": ["runtime device copy", "elementwise y = x + 0"]}


KERNEL_SOURCES = ("likelihood.hip", "kernels.hip", "rbl_launch.h", "rbl_internal.h", "rbl_wave.h", "rbl_math.h", "rbl_phasor.h",
                  "rbl_physics.h", "rbl_nrtv2.h")


def kernel_source_hash():
    """sha256 over the code of the kernel sources (line comments and blank lines removed, so
    that a comment edit keeps the hash): counters taken on other code do not apply."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2404_11397_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"\s*//.*$", "", line.rstrip("\n")).rstrip()
                if code:
                    h.update(code.encode("utf-8") + b"\n")
    return h.hexdigest()[:16]


def stored_traffic(kernel_tag):
    """HBM bytes per launch of a kernel from the committed counter summary
    profiles/<kernel_tag>_traffic.md (a line 'traffic: {json}'), if it was taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic: "):
                rec = json.loads(line[len("traffic: "):])
                return rec if rec.get("source_hash") == kernel_source_hash() else None
    return None


def forms_on(torch, ev, theta, lnl, grad, ws, steps, with_grad=True):
    """evals/s and HIP-event kernel times of lnL and lnL+grad, FP64 and mixed."""
    B = theta.shape[0]
    out = {}
    combos = [("lnl", False), ("lnl_grad", True)] if with_grad else [("lnl", False)]
    for tag, g in combos:
        for prec in ("fp64", "mixed"):
            if g:
                fn = lambda p=prec: ev.loglike_grad(theta, p, out=(lnl, grad), workspace=ws)  # noqa: E731
            else:
                fn = lambda p=prec: ev.loglike(theta, p, out=lnl[:B], workspace=ws)  # noqa: E731
            el, ku, su = time_calls(torch, fn, steps, 3)
            out[f"{tag}_{prec}"] = {"evals_per_s": B * steps / el, "us_per_call": el / steps * 1e6,
                                    "kernel_us": ku, "setup_us": su}
    return out


def nrtv2_forms(torch, steps):
    """IMRPhenomD_NRTidalv2 on the 3-detector 256 s data: lnL+grad at 8192 chains and
    lnL at 16384 chains, FP64 and mixed, with the estimated VALU fraction."""
    ev, w, edges, data = build_event(torch, "nrtv2_3det_256s_grad8192")
    nd, n_nodes = len(w["tensors"]), w["n_bins"] + 1
    res = {"workload": "IMRPhenomD_NRTidalv2: 3 det, 256 s, 20-2048 Hz (519169 pts/det), 1000 bins, SNR 12 "
                       "injection; lnL+grad at 8192 chains (GW190425 prior, Mc window +-0.0025), lnL at 16384"}
    th = torch.as_tensor(w["theta"], device="cuda:0")
    B = th.shape[0]
    lnl = torch.empty(2 * B, dtype=torch.float64, device="cuda:0")
    grad = torch.empty((B, 13), dtype=torch.float64, device="cuda:0")
    ws = ev.workspace(2 * B, with_grad=True)
    f = forms_on(torch, ev, th, lnl[:B], grad, ws, steps)
    w3 = synth.workload("nrtv2_3det_256s")
    th3 = torch.as_tensor(w3["theta"], device="cuda:0")
    f.update({k + "_16384": v for k, v in forms_on(torch, ev, th3, lnl, grad, ws, steps, with_grad=False).items()})
    for k, v in f.items():
        g = "grad" in k
        per, _ = flops_per_eval(n_nodes, nd, grad=g, waveform="phenomd_nrtv2")
        nb = th3.shape[0] if k.endswith("16384") else B
        v["est_tflops"] = per * nb / (v["kernel_us"] * 1e-6) / 1e12
        v["est_frac_fp64_peak"] = v["est_tflops"] / PEAK_FP64_TFLOPS
    psd = torch.as_tensor(w["psd"], device="cuda:0")
    su = summary_pass(torch, w, edges, data, psd)
    nbytes = w["n_freq"] * nd * 24
    res["forms"] = f
    res["summary_pass"] = {"us": su, "bytes": nbytes, "GB_per_s": nbytes / (su * 1e-6) / 1e9,
                           "frac_of_hbm_peak": nbytes / (su * 1e-6) / 1e9 / PEAK_HBM_GBS}
    return res


def build_serving_events(torch):
    """The 64 serving events.  An IMRPhenomD_NRTidalv2 event whose untapered reference
    amplitude reaches zero inside the band (large tidal deformabilities: the tidal
    amplitude correction outgrows the point-particle amplitude) is rejected by the
    library (RBL_EREF); its injection then has Lambda1 and Lambda2 halved until the
    reference is valid.  Returns the events, their theta pools, specs and the number
    of events so adjusted."""
    from paper_2404_11397_amd import Event, RblError, bin_edges, strain
    events, pools, specs = [], [], []
    adjusted = 0
    dev = torch.device("cuda:0")
    for eid in range(synth.N_SERVE_EVENTS):
        sp = synth.serving_event(eid)
        x = synth.serving_inputs(sp)
        edges = bin_edges(x["f_low"], x["delta_f"], x["n_freq"], sp["n_bins"])
        psd = torch.as_tensor(x["psd"], device=dev)
        noise = torch.as_tensor(x["noise"], device=dev)
        th = sp["theta_inj"].copy()
        for attempt in range(12):
            h = strain(sp["waveform"], x["tensors"], x["vertices"], sp["gmst"], x["f_low"], x["delta_f"],
                       x["n_freq"], th, device=dev)
            try:
                ev = Event(h + noise, psd, x["tensors"], x["vertices"], sp["gmst"], x["f_low"], x["delta_f"], th,
                           edges, waveform=sp["waveform"], device=dev)
                break
            except RblError as e:
                if e.code != -6 or sp["waveform"] != "phenomd_nrtv2" or attempt == 11:
                    raise
                th[4] *= 0.5
                th[5] *= 0.5
        adjusted += int(attempt > 0)
        sp["theta_inj"] = th
        events.append(ev)
        pools.append([np.ascontiguousarray(p) for p in x["pool"]])
        specs.append(sp)
        del h, psd, noise
    return events, pools, specs, adjusted


def run_stream(srv, ids, pools, n, rate, precision):
    """Submit n requests at Poisson arrival times; latency = done - arrival (host clock)."""
    import queue
    import threading
    from paper_2404_11397_amd import clock_ns
    offs, evs, pidx = synth.serving_stream(n, rate)
    q = queue.Queue()
    lat = np.empty(n)
    wait_adm = np.empty(n)
    done = np.empty(n, dtype=np.int64)
    chains = np.array([pools[e][k].shape[0] for e, k in zip(evs, pidx)])

    def waiter():
        for i in range(n):
            _, _, info = srv.wait(q.get())
            lat[i] = (info["t_done_ns"] - info["t_arrival_ns"]) * 1e-6
            wait_adm[i] = (info["t_admit_ns"] - info["t_arrival_ns"]) * 1e-6
            done[i] = info["t_done_ns"]

    th = threading.Thread(target=waiter)
    th.start()
    t0 = clock_ns() + 5_000_000
    for i in range(n):
        ta = t0 + int(offs[i] * 1e9)
        while True:
            d = ta - clock_ns()
            if d <= 0:
                break
            if d > 400_000:
                time.sleep((d - 300_000) * 1e-9)
        q.put(srv.submit(ids[evs[i]], pools[evs[i]][pidx[i]], precision=precision, grad=True, t_arrival_ns=ta))
    th.join()
    span = (done.max() - t0) * 1e-9
    return {"rate_hz": rate, "requests": n, "precision": precision,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "admit_wait_p50_ms": float(np.percentile(wait_adm, 50)),
            "service_p50_ms": float(np.percentile(lat - wait_adm, 50)), "evals_per_s": float(chains.sum() / span),
            "offered_evals_per_s": float(chains.sum() / (offs[-1] + 1e-9))}


def serving(torch, n_requests):
    """The multi-event request stream: 64 resident events, Poisson arrivals, lnL+grad
    per request.  Served by the library's request server (mixed precision, 4 streams,
    graph replays) and, for comparison, one FIFO with FP64 plain launches."""
    from paper_2404_11397_amd import Server
    t_build = time.perf_counter()
    events, pools, specs, adjusted = build_serving_events(torch)
    t_build = time.perf_counter() - t_build
    budget = 32 << 30
    res = {"workload": f"{synth.N_SERVE_EVENTS} resident events (1-3 det, 32-256 s, 100-1000 bins, TaylorF2 / "
                       f"IMRPhenomD_NRTidalv2, 256-4096 chains each); Poisson {synth.SERVE_RATE_HZ:.0f} req/s of "
                       "lnL+grad requests",
           "events_build_s": t_build, "hbm_budget_bytes": budget,
           "nrtv2_events_with_halved_lambda": adjusted}
    for tag, streams, graphs, spin, prec in (("server", 4, True, True, "mixed"),
                                             ("baseline_fifo_fp64_plain", 1, False, False, "fp64")):
        with Server(budget, n_streams=streams, graphs=graphs, spin=spin) as srv:
            ids = [srv.add_event(e) for e in events]
            warm = [srv.submit(ids[e], pools[e][k], precision=prec) for e in range(len(events))
                    for k in range(len(pools[e]))]
            for t in warm:
                srv.wait(t)
            r = run_stream(srv, ids, pools, n_requests, synth.SERVE_RATE_HZ, prec)
            r["saturation"] = [run_stream(srv, ids, pools, n_requests, rate, prec) for rate in (2000.0, 20000.0)]
            r["stats"] = srv.stats()
            r["streams"], r["graphs"], r["spin"] = streams, graphs, spin
            res[tag] = r
    res["resident_bytes"] = res["server"]["stats"]["resident_bytes"]
    return res


def mala_rate(torch, ev, w, steps):
    """Device MALA local steps (proposal, lnL+grad, accept) on the headline event: chain-steps/s.

    Chains start around the injection with the spread of a diagonal Fisher estimate
    (sigma_i = 1 / rms of dlnL/dz_i at the injection, i.e. inverse-Fisher), the step is
    s_i = (f sigma_i)^2, and f is adapted during the untimed warm-up towards an acceptance
    of about 0.6; the timed steps keep f fixed."""
    from paper_2404_11397_amd import Mala
    th0 = w["theta_inj"]
    z0 = th0.copy()
    z0[9] = np.cos(th0[9])
    z0[12] = np.sin(th0[12])
    B = len(w["theta"])
    b = synth.PRIORS["gw170817"]
    lo = np.array([b["Mc"][0], b["q"][0], b["chi"][0], b["chi"][0], b["L"][0], b["L"][0], b["dL"][0], b["tc"][0],
                   0.0, -1.0, 0.0, 0.0, -1.0])
    hi = np.array([b["Mc"][1], b["q"][1], b["chi"][1], b["chi"][1], b["L"][1], b["L"][1], b["dL"][1], b["tc"][1],
                   2 * np.pi, 1.0, np.pi, 2 * np.pi, 1.0])
    rng = np.random.default_rng(77)
    probe = np.clip(z0 + 1e-7 * (hi - lo) * rng.standard_normal((B, 13)), lo, hi)
    g = Mala(ev, torch.as_tensor(probe, device="cuda:0")).gz.cpu().numpy()
    sigma = 1.0 / np.sqrt(np.mean(g * g, axis=0) + 1e-300)
    sigma = np.minimum(sigma, 0.05 * (hi - lo))
    start = np.clip(z0 + sigma * rng.standard_normal((B, 13)), lo, hi)
    ch = Mala(ev, torch.as_tensor(start, device="cuda:0"))
    gen = torch.Generator(device="cuda:0").manual_seed(7)
    f = 0.5
    for _ in range(30):
        xi = torch.randn((B, 13), dtype=torch.float64, device="cuda:0", generator=gen)
        logu = torch.log(torch.rand(B, dtype=torch.float64, device="cuda:0", generator=gen))
        a = float(ch.step((f * sigma) ** 2, lo, hi, xi, logu).double().mean())
        f *= 1.3 if a > 0.6 else 0.7
    step = (f * sigma) ** 2
    xi = torch.randn((steps, B, 13), dtype=torch.float64, device="cuda:0", generator=gen)
    logu = torch.log(torch.rand((steps, B), dtype=torch.float64, device="cuda:0", generator=gen))
    acc = torch.zeros(B, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        acc += ch.step(step, lo, hi, xi[k], logu[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"chain_steps_per_s": B * steps / dt, "us_per_step": dt / steps * 1e6, "chains": B, "steps": steps,
            "acceptance": float(acc.sum()) / (B * steps), "step_factor": f, "precision": "fp64",
            "what": "rbl_mala_step on the headline event (proposal, setup + lnL+grad kernels, accept), chains "
                    "around the injection, diagonal inverse-Fisher preconditioning, step adapted in warm-up"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the likelihood shards over "
                                   "chains with no exchange, so no multi-GPU figure is measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    workload = "tf2_3det_128s_grad8192"
    ev, w, edges, data = build_event(torch, workload)
    theta_np = w["theta"]
    B = theta_np.shape[0]
    theta = torch.as_tensor(theta_np, device="cuda:0")
    lnl = torch.empty(B, dtype=torch.float64, device="cuda:0")
    grad = torch.empty((B, 13), dtype=torch.float64, device="cuda:0")
    ws = ev.workspace(B, with_grad=True)

    def step():
        ev.loglike_grad(theta, args.precision, out=(lnl, grad), workspace=ws)

    elapsed, kern_us, setup_us = time_calls(torch, step, args.steps, args.warmup)

    # per-call latency of a synchronised batch call
    lat = []
    for _ in range(50):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)

    forms = forms_on(torch, ev, theta, lnl, grad, ws, max(20, args.steps // 4))

    nd = len(w["tensors"])
    psd = torch.as_tensor(w["psd"], device="cuda:0")
    summ_us = summary_pass(torch, w, edges, data, psd)
    summ_bytes = w["n_freq"] * nd * 24  # data (complex128) + PSD (float64) per grid point and detector

    n_nodes = w["n_bins"] + 1
    fl_kernel, _ = flops_per_eval(n_nodes, nd, grad=True)
    achieved = fl_kernel * B / (kern_us * 1e-6) / 1e12
    out = {
        "metric": "relative-binned lnL+grad evals/sec (13-param BNS, 3 det); p50/p99 latency",
        "value": B * args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64-phase/f32",
        "data": "synthetic (library waveform injections + seeded Gaussian noise, analytic PSD)",
        "config": {"workload": "TaylorF2 lnL+grad: 3 det, 128 s, 20-2048 Hz (259585 pts/det), "
                               "500 bins, 8192 chains, GW170817 prior",
                   "global_batch": B, "n_bins": w["n_bins"], "n_det": nd, "n_freq": w["n_freq"],
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_loglike_grad<3>", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None, "flops_per_eval": fl_kernel,
                     "avg_kernel_us": kern_us, "avg_setup_us": setup_us,
                     "kernel_timing": f"HIP start/stop events on the kernel's own stream, on the first and every "
                                      f"{TIMING_EVERY}th call of the timed region",
                     "kernel_source_hash": kernel_source_hash()},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one synchronised rbl_loglike_grad call over the 8192-chain batch"},
        "forms": forms,
        "summary_pass": {"us": summ_us, "bytes": summ_bytes, "GB_per_s": summ_bytes / (summ_us * 1e-6) / 1e9,
                         "frac_of_hbm_peak": summ_bytes / (summ_us * 1e-6) / 1e9 / PEAK_HBM_GBS},
    }
    out["mala"] = mala_rate(torch, ev, w, max(20, args.steps // 4))
    out["full_band"] = full_band(torch, max(10, args.steps // 10))
    tr = stored_traffic("k_loglike_grad_tf2_3det_128s_8192_fp64")
    if tr is not None:
        out["roofline"]["traffic"] = tr["hbm_bytes_per_launch"]
        out["roofline"]["traffic_detail"] = tr
    if not args.no_nrtv2:
        out["nrtv2"] = nrtv2_forms(torch, max(20, args.steps // 4))
    if not args.no_serve:
        sv = serving(torch, args.serve_requests)
        out["serving"] = sv
        out["latency_ms"] = {"p50": sv["server"]["p50_ms"], "p99": sv["server"]["p99_ms"],
                             "what": "request latency (arrival to results in host memory) under the "
                                     "multi-event Poisson stream, request server",
                             "batch_call_p50": float(np.percentile(lat, 50)),
                             "batch_call_p99": float(np.percentile(lat, 99))}
    if args.calibrate_copy:
        out["copy_calibration"] = calibrate_copy(torch)
    if not args.no_cpu_baseline:
        data_host = data.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(w, edges, data_host, theta_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
