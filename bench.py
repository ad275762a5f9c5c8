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
NRTV2_NOTE = ("unpinned: IMRPhenomD_NRTidalv2 here is a structural stand-in (the published calibration "
              "tables are not available); GPU parity is against the oracle's identical stand-in")
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


def flops_mixed_split(n_nodes, n_det, grad, waveform="taylorf2"):
    """(FP64, FP32) flops per eval of the mixed form, the split of the same operations as
    flops_per_eval: FP64 keeps the edge phase (TaylorF2 basis 28 / IMRPhenomD_NRTidalv2 node
    model 110), per detector the delay term (2), the exact reduction to revolutions (2) and
    the FP64 accumulation of the per-edge terms (4; gradient 6 more), the gradient's basis or
    node-parameter accumulations (20 / 180) and the per-chain setup; FP32 takes per detector
    the hardware sin/cos (two quarter-rate instructions: 8), the ratio (6; NRTidalv2 + 2 for
    the amplitude ratio) and the remaining binned products (10; gradient 20)."""
    amp = 0 if waveform == "taylorf2" else 2
    f64 = (28 if waveform == "taylorf2" else 110) + n_det * (2 + 2 + 4)
    f32 = n_det * (8 + 6 + amp + 10)
    if grad:
        f64 += (20 if waveform == "taylorf2" else 180) + 6 * n_det
        f32 += 20 * n_det
    _, setup = flops_per_eval(n_nodes, n_det, grad, waveform)
    return n_nodes * f64, n_nodes * f32, setup


PEAK_FP32_TFLOPS = 157.3


def mixed_roofline(n_nodes, n_det, grad, waveform, chains, kernel_us):
    """Roofline of a mixed-form kernel: t_bound = F64 / P64 + F32 / P32 for its modelled
    flop split; frac = t_bound / measured kernel time."""
    f64, f32, _ = flops_mixed_split(n_nodes, n_det, grad, waveform)
    t_bound = chains * (f64 / (PEAK_FP64_TFLOPS * 1e12) + f32 / (PEAK_FP32_TFLOPS * 1e12))
    return {"f64_flops_per_eval": f64, "f32_flops_per_eval": f32, "t_bound_us": t_bound * 1e6,
            "frac": t_bound / (kernel_us * 1e-6)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
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


def _oracle_event(workload):
    """The workload's event built entirely by the oracle (its own injection and bins)."""
    from oracle import binning
    from oracle import likelihood as L
    from oracle import waveform as W
    w = synth.workload(workload)
    ev = L.Event(f=w["f"], delta_f=w["delta_f"], psd=w["psd"], data=None, tensors=w["tensors"],
                 vertices=w["vertices"], gmst=w["gmst"], approximant=w["waveform"])
    h = W.strain(w["f"], w["theta_inj"], w["tensors"], w["vertices"], w["gmst"], w["waveform"], True)
    ev.data = np.stack([x[0] for x in h]) + w["noise"]
    ev.theta_ref = w["theta_inj"]
    ev.edges = binning.pn_bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"])
    L.prepare(ev)
    return ev, w["theta"]


_CPU = {}
CPU_CHUNK = 32


def _cpu_worker(args):
    """Oracle lnL + dual-number gradient on chunks of the batch for `seconds` (one process)."""
    from oracle import likelihood as L
    offset, seconds = args
    ev, theta = _CPU["ev"], _CPU["theta"]
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        lo = (offset + done) % (len(theta) - CPU_CHUNK)
        L.loglike_rb_grad(ev, theta[lo:lo + CPU_CHUNK])
        done += CPU_CHUNK
    return done, time.perf_counter() - t0


def cpu_baseline(workload, seconds):
    """The FP64 oracle (lnL + dual-number gradient) timed on a bounded sample of the workload:
    once in one process, once in a pool of processes over the host cores this job may use
    (at most 16, the host share of one GPU).  Runs before the GPU is initialised, on the
    oracle's own injection of the same workload (its timing does not depend on the data)."""
    import multiprocessing as mp
    _CPU["ev"], _CPU["theta"] = _oracle_event(workload)
    one, dt1 = _cpu_worker((0, seconds))
    cores = max(1, min(len(os.sched_getaffinity(0)), 16))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(k * 997, seconds) for k in range(cores)])
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    return {"value": total / wall, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{total} chain evaluations (lnL + dual-number gradient, chunks of {CPU_CHUNK} chains cycling "
                      f"through the {workload} batch) in {wall:.1f} s by {cores} processes of numpy FP64, one "
                      f"thread each",
            "single_core": {"value": one / dt1, "unit": "evals/s", "cores": 1,
                            "sample": f"{one} chain evaluations in {dt1:.1f} s, one process"}}


KERNEL_PASS_CALLS = 50  # calls of the separate pass that takes the kernel times
# The GPU raises its clocks over the first ~30 ms of back-to-back work and lowers them again
# when idle (measured on the headline step: 78, 46, 44, 43, 42, 41 us per step over the first
# six chunks of 100 calls, 41 us from there on, and 47 us again after two idle seconds).  Every
# timed region is therefore preceded by untimed calls until this much time has passed, so that
# it measures the steady state of a sampler that keeps the device busy.
CLOCK_RAMP_S = 0.3


def ramp(torch, fn, warmup, ramp_fn=None, seconds=CLOCK_RAMP_S):
    """The untimed calls before a timed region: calls of ramp_fn (default: fn) until `seconds`
    of back-to-back work have passed (the host waits for the device every 16 calls, so that it
    never runs far ahead), then `warmup` calls of fn, with no pause in between.  Returns
    (calls, seconds)."""
    rf = ramp_fn or fn
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        rf()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    return n + warmup, time.perf_counter() - t0


LAST_RAMP = {}


def time_calls(torch, fn, steps, warmup, ramp_fn=None):
    """Wall time of `steps` calls (no kernel timing inside the timed region) after the
    untimed ramp, then the average kernel durations (main, setup) [us] from a separate pass
    of min(steps, KERNEL_PASS_CALLS) calls, each stamped with HIP start/stop events that the
    runtime records at the kernels' own start and end on the launch stream.  A call that
    changes state (a sampler step) passes a ramp_fn that does not."""
    from paper_2404_11397_amd import profile_enable, profile_read
    n, dt = ramp(torch, fn, warmup, ramp_fn)
    LAST_RAMP.update(calls=n, seconds=dt)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    profile_enable(True, every=1)
    for _ in range(min(steps, KERNEL_PASS_CALLS)):
        fn()
    torch.cuda.synchronize()
    main_ms, setup_ms, calls = profile_read()
    profile_enable(False)
    return elapsed, main_ms / calls * 1e3, setup_ms / calls * 1e3


def full_flops(n_freq, chains, n_det, waveform="taylorf2"):
    """Algorithmic FP64 flops of a full-band lnL batch (Eqs. (2)-(3) on every grid point).
    Per grid point, shared by the batch: x = f^(1/3) (20), 1/x (10), ln x (20), f^(-7/6) (23),
    the TaylorF2 basis (8) or x^5.78 (20 + 1), and per detector 1/S (10).  Per point and
    chain: the TaylorF2 basis phase (20) or the IMRPhenomD_NRTidalv2 node model (110) and its
    amplitude factor (1); per detector the phase with delay (2), sin/cos of a phase in
    revolutions (36), the strain (8) and the two inner-product terms with their weight and
    sum (10)."""
    if waveform == "taylorf2":
        shared, per_chain = 81 + 10 * n_det, 20 + 56 * n_det
    else:
        shared, per_chain = 94 + 10 * n_det, 111 + 56 * n_det
    return n_freq * shared + n_freq * chains * per_chain


def diag_information_sigma(grad_fn, x0, widths, cap):
    """sigma_i = 1 / sqrt(I_ii) with I_ii = -d^2 lnL / dx_i^2 at x0, the diagonal of the
    observed information, by central differences of the library gradient with steps
    h_i = 1e-6 of the prior widths; components with I_ii <= 0 or a sigma above `cap` take
    `cap`.  grad_fn: [n, 13] -> [n, 13] (numpy)."""
    h = 1e-6 * widths
    probes = np.repeat(x0[None, :], 26, axis=0)
    for i in range(13):
        probes[2 * i, i] += h[i]
        probes[2 * i + 1, i] -= h[i]
    g = grad_fn(probes)
    info = np.array([-(g[2 * i, i] - g[2 * i + 1, i]) / (2 * h[i]) for i in range(13)])
    sigma = np.where(info > 0, 1.0 / np.sqrt(np.maximum(info, 1e-300)), np.inf)
    return np.minimum(sigma, cap)


def _near_draws(ev, w, B, rng):
    """B draws around the injection with spreads 1/sqrt(-d2 lnL/dtheta_i2) there (the diagonal
    of the observed information, from the library gradient)."""
    th0 = w["theta_inj"]
    sigma = diag_information_sigma(
        lambda x: ev.loglike_grad(torch_mod().as_tensor(x, device="cuda:0"))[1].cpu().numpy(), th0, WIDTHS,
        0.05 * np.abs(th0) + 1e-3)
    near = th0 + sigma * rng.standard_normal((B, 13))
    near[:, 1] = np.clip(near[:, 1], 0.05, 1.0)
    near[:, 2:4] = np.clip(near[:, 2:4], -0.99, 0.99)
    near[:, 4:6] = np.maximum(near[:, 4:6], 0.0)
    near[:, 9] = np.clip(near[:, 9], 1e-3, np.pi - 1e-3)
    near[:, 12] = np.clip(near[:, 12], -np.pi / 2 + 1e-3, np.pi / 2 - 1e-3)
    return near


def torch_mod():
    import torch
    return torch


FULL_BAND_CASES = (("tf2_1det_32s", 256, None), ("tf2_3det_128s", 4096, None), ("nrtv2_3det_256s", 1024, 2048))


def full_band(torch, steps):
    """Full-band lnL (every grid point, no binning) beside the binned FP64 lnL on the same batch,
    on the 1-detector 32 s, 3-detector 128 s and 3-detector 256 s workloads: throughput, the
    full-band kernel against its roofline, and the binning error of Eq. (5) over each
    workload's prior draws and around its injection."""
    out = {}
    for name, B, B_err in FULL_BAND_CASES:
        ev, w, edges, data = build_event(torch, name, keep_grid=True)
        nd = len(w["tensors"])
        th_all = torch.as_tensor(w["theta"], device="cuda:0")
        th = th_all[:B].contiguous()
        ws = ev.workspace(max(B, B_err or 0), False)
        full = torch.empty(B, dtype=torch.float64, device="cuda:0")
        rb = torch.empty_like(full)
        n_steps = steps if nd == 1 else max(3, steps // 4)
        el_f, ku_f, su_f = time_calls(torch, lambda: ev.loglike_full(th, out=full, workspace=ws[:ev.workspace_bytes(B)]),
                                      n_steps, 2)
        el_b, ku_b, su_b = time_calls(torch, lambda: ev.loglike(th, out=rb, workspace=ws[:ev.workspace_bytes(B)]),
                                      n_steps, 2)
        fl = full_flops(w["n_freq"], B, nd, w["waveform"])
        # binning error over the workload's prior draws and around the injection
        the = th_all[:B_err].contiguous() if B_err else th
        err_p = (ev.loglike(the) - ev.loglike_full(the)).abs()
        near = torch.as_tensor(_near_draws(ev, w, min(B, 1024), np.random.default_rng(91)), device="cuda:0")
        full_n = ev.loglike_full(near)
        err_n = (ev.loglike(near) - full_n).abs()
        out[name] = {
            "workload": f"{w['waveform']}, {nd} det, {w['duration']:.0f} s, {w['n_freq']} points per detector, "
                        f"{w['n_bins']} bins, {B} chains",
            "full_evals_per_s": B * n_steps / el_f, "full_kernel_us": ku_f, "full_setup_us": su_f,
            "roofline": {"bound": "alu", "achieved": fl / (ku_f * 1e-6) / 1e12, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": fl / (ku_f * 1e-6) / 1e12 / PEAK_FP64_TFLOPS,
                         "flops_per_launch": fl, "kernel": "k_full_tiles"},
            "binned_evals_per_s": B * n_steps / el_b, "binned_kernel_us": ku_b, "kernel_speedup": ku_f / ku_b,
            "binning_error_prior_draws": {
                "chains": int(the.shape[0]), "max_abs": float(err_p.max()), "median_abs": float(err_p.median()),
                "what": "the workload's prior draws; far from the reference the linear model of Eq. (5) is not "
                        "meant to hold"},
            "binning_error_near_injection": {
                "chains": int(near.shape[0]), "max_abs": float(err_n.max()), "median_abs": float(err_n.median()),
                "lnl_range": [float(full_n.min()), float(full_n.max())],
                "what": "draws around the injection with spreads 1/sqrt(-d2 lnL/dtheta_i2) there (diagonal of the "
                        "observed information, central differences of the library gradient)"}}
        del ev, data
        progress(f"full band {name} done")
    return out


def reference_search(torch, n_starts=16, lam=128, generations=400):
    """The CMA-ES reference-parameter search (rbl_ref_search) on a noise-free injection into the
    3-detector 128 s TaylorF2 workload, over the GW170817 prior box: n_starts runs from points
    drawn uniformly over the box, advanced together.  Wall time, candidate evaluations per
    second, how far below the peak (<h, h>/2 at the injection) the best candidate ends, and how
    many runs end within 13/2 of it."""
    from paper_2404_11397_amd import Event, bin_edges, ref_search, strain
    w = synth.workload("tf2_3det_128s", batch=1)
    dev = torch.device("cuda:0")
    th0 = w["theta_inj"]
    h = strain("taylorf2", w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"], w["n_freq"], th0,
               device=dev)
    ev = Event(h, torch.as_tensor(w["psd"], device=dev), w["tensors"], w["vertices"], w["gmst"], w["f_low"],
               w["delta_f"], th0, bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"]), keep_grid=True,
               device=dev)
    b = synth.PRIORS["gw170817"]
    lo = np.array([b["Mc"][0], b["q"][0], b["chi"][0], b["chi"][0], b["L"][0], b["L"][0], b["dL"][0], b["tc"][0],
                   0.0, 0.0, 0.0, 0.0, -np.pi / 2])
    hi = np.array([b["Mc"][1], b["q"][1], b["chi"][1], b["chi"][1], b["L"][1], b["L"][1], b["dL"][1], b["tc"][1],
                   2 * np.pi, np.pi, np.pi, 2 * np.pi, np.pi / 2])
    rng = np.random.default_rng(21)
    starts = lo + rng.random((n_starts, 13)) * (hi - lo)
    normals = rng.standard_normal((n_starts, generations, lam, 13))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best, best_l, traces = ref_search(ev, lo, hi, starts, 0.3, normals)
    dt = time.perf_counter() - t0
    peak = float(ev.loglike_full(torch.as_tensor(th0[None, :], device=dev))[0])
    finals = np.array([t[-1, 0] for t in traces])
    evals = lam * sum(len(t) for t in traces)
    return {"workload": "noise-free TaylorF2 injection, 3 det, 128 s, 259585 points per detector; GW170817 prior box, "
                        f"{n_starts} starts drawn uniformly over it",
            "n_starts": n_starts, "lambda": lam, "generations": generations,
            "generations_run": [len(t) for t in traces], "seconds": dt, "candidate_evals_per_s": evals / dt,
            "lnl_peak": peak, "lnl_found": best_l, "delta_lnl": peak - best_l,
            "runs_within_6.5_of_peak": int(np.sum(peak - finals <= 6.5)),
            "delta_lnl_per_run": (peak - finals).tolist(),
            "found_minus_injection": (best - th0).tolist(),
            "what": "rbl_ref_search: CMA-ES runs over the full-band lnL, the populations of all runs evaluated "
                    "together on the device each generation, updates on the host"}


def summary_pass(torch, w, edges, data, psd, repeats=5, ramp_fn=None):
    """Average duration of the summary-data kernel of rbl_event_create (HIP events), over
    `repeats` event builds after one untimed build.  With ramp_fn (device work), the builds run
    at the clocks of sustained work: the clock ramp first, and 30 ms of ramp_fn calls before
    each build."""
    from paper_2404_11397_amd import Event, profile_enable, profile_read_summary
    if ramp_fn is not None:
        ramp(torch, ramp_fn, 0)
    Event(data, psd, w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"], w["theta_inj"], edges,
          waveform=w["waveform"], device=data.device)
    profile_enable(True)
    profile_read_summary()
    for _ in range(repeats):
        if ramp_fn is not None:
            ramp(torch, ramp_fn, 0, seconds=0.03)
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


WIDTHS = np.array([0.03, 0.875, 0.1, 0.1, 5000.0, 5000.0, 74.0, 0.2, 2 * np.pi, np.pi, np.pi, 2 * np.pi, np.pi])


def mixed_error(torch, ev, theta, with_grad):
    """The mixed form against the FP64 form on the same batch (the FP64 GPU path is the
    oracle-pinned one): max and median |dlnL|, the largest prior-width-scaled gradient error
    relative to the chain's largest scaled component, and the chains the mixed form's guard
    computed in FP64 (results bitwise equal to the FP64 ones)."""
    if with_grad:
        l64, g64 = (x.clone() for x in ev.loglike_grad(theta, "fp64"))
        l32, g32 = ev.loglike_grad(theta, "mixed")
    else:
        l64, l32 = ev.loglike(theta, "fp64").clone(), ev.loglike(theta, "mixed")
    d = (l32 - l64).abs()
    ok = torch.isfinite(d)
    out = {"max_abs_dlnl": float(d[ok].max()), "median_abs_dlnl": float(d[ok].median()),
           "chains": int(theta.shape[0]), "chains_guarded_to_fp64": int((l32 == l64).sum())}
    if with_grad:
        w = torch.as_tensor(WIDTHS, device=theta.device)
        gs, ws = g32 * w, g64 * w
        rel = (gs - ws).abs().max(dim=1).values / ws.abs().max(dim=1).values
        out["max_grad_rel_err"] = float(rel[torch.isfinite(rel)].max())
    return out


def forms_on(torch, ev, theta, lnl, grad, ws, steps, with_grad=True, n_nodes=None, n_det=None,
             waveform="taylorf2"):
    """evals/s and kernel times of lnL and lnL+grad, FP64 and mixed; for the mixed rows
    the error against FP64 and the mixed-form roofline."""
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
            row = {"evals_per_s": B * steps / el, "us_per_call": el / steps * 1e6, "kernel_us": ku, "setup_us": su}
            if prec == "mixed":
                row["error_vs_fp64"] = mixed_error(torch, ev, theta, g)
                if n_nodes is not None:
                    row["roofline_mixed"] = mixed_roofline(n_nodes, n_det, g, waveform, B, ku)
            out[f"{tag}_{prec}"] = row
    return out


def nrtv2_forms(torch, steps):
    """IMRPhenomD_NRTidalv2 on the 3-detector 256 s data: lnL+grad at 8192 chains and
    lnL at 16384 chains, FP64 and mixed, with the estimated VALU fraction."""
    ev, w, edges, data = build_event(torch, "nrtv2_3det_256s_grad8192")
    nd, n_nodes = len(w["tensors"]), w["n_bins"] + 1
    res = {"workload": "IMRPhenomD_NRTidalv2: 3 det, 256 s, 20-2048 Hz (519169 pts/det), 1000 bins, SNR 12 "
                       "injection; lnL+grad at 8192 chains (GW190425 prior, Mc window +-0.0025), lnL at 16384",
           "parity_vs_published_model": NRTV2_NOTE}
    th = torch.as_tensor(w["theta"], device="cuda:0")
    B = th.shape[0]
    lnl = torch.empty(2 * B, dtype=torch.float64, device="cuda:0")
    grad = torch.empty((B, 13), dtype=torch.float64, device="cuda:0")
    ws = ev.workspace(2 * B, with_grad=True)
    f = forms_on(torch, ev, th, lnl[:B], grad, ws, steps, n_nodes=n_nodes, n_det=nd, waveform="phenomd_nrtv2")
    w3 = synth.workload("nrtv2_3det_256s")
    th3 = torch.as_tensor(w3["theta"], device="cuda:0")
    f.update({k + "_16384": v for k, v in forms_on(torch, ev, th3, lnl, grad, ws, steps, with_grad=False,
                                                    n_nodes=n_nodes, n_det=nd, waveform="phenomd_nrtv2").items()})
    for k, v in f.items():
        g = "grad" in k
        per, _ = flops_per_eval(n_nodes, nd, grad=g, waveform="phenomd_nrtv2")
        nb = th3.shape[0] if k.endswith("16384") else B
        v["est_tflops"] = per * nb / (v["kernel_us"] * 1e-6) / 1e12
        v["est_frac_fp64_peak"] = v["est_tflops"] / PEAK_FP64_TFLOPS
    psd = torch.as_tensor(w["psd"], device="cuda:0")
    su = summary_pass(torch, w, edges, data, psd, ramp_fn=lambda: ev.loglike(th, out=lnl[:B], workspace=ws))
    nbytes = w["n_freq"] * nd * 24
    res["forms"] = f
    res["summary_pass"] = {"us": su, "bytes": nbytes, "GB_per_s": nbytes / (su * 1e-6) / 1e9,
                           "frac_of_hbm_peak": nbytes / (su * 1e-6) / 1e9 / PEAK_HBM_GBS}
    return res


def build_serving_events(torch):
    """The 64 serving events with their configured injections (library waveform + seeded
    noise).  An IMRPhenomD_NRTidalv2 event whose untapered reference amplitude reaches zero
    inside 20-2048 Hz is refused by the library (RBL_EREF: the ratio of Eq. (4) is undefined
    there); it is analysed on a band that ends at the last grid point where the tapered
    injection is non-zero, just below the end of the reference's taper (1.2 f_merger), with
    its bins placed on that band.  Returns the events, their theta pools, specs and the
    {event id: band end [Hz]} of the events so cut."""
    from paper_2404_11397_amd import Event, RblError, bin_edges, strain
    events, pools, specs = [], [], []
    cuts = {}
    dev = torch.device("cuda:0")
    for eid in range(synth.N_SERVE_EVENTS):
        sp = synth.serving_event(eid)
        x = synth.serving_inputs(sp)
        n = x["n_freq"]
        psd = torch.as_tensor(x["psd"], device=dev)
        noise = torch.as_tensor(x["noise"], device=dev)
        th = sp["theta_inj"]
        h = strain(sp["waveform"], x["tensors"], x["vertices"], sp["gmst"], x["f_low"], x["delta_f"], n, th,
                   device=dev)
        try:
            ev = Event(h + noise, psd, x["tensors"], x["vertices"], sp["gmst"], x["f_low"], x["delta_f"], th,
                       bin_edges(x["f_low"], x["delta_f"], n, sp["n_bins"]), waveform=sp["waveform"], device=dev)
        except RblError as e:
            if e.code != -6 or sp["waveform"] != "phenomd_nrtv2":
                raise
            n = int(torch.nonzero((h.abs() > 0).any(dim=0))[-1]) + 1
            cuts[eid] = x["f_low"] + (n - 1) * x["delta_f"]
            ev = Event((h + noise)[:, :n], psd[:, :n], x["tensors"], x["vertices"], sp["gmst"], x["f_low"],
                       x["delta_f"], th, bin_edges(x["f_low"], x["delta_f"], n, sp["n_bins"]),
                       waveform=sp["waveform"], device=dev)
        events.append(ev)
        pools.append([np.ascontiguousarray(p) for p in x["pool"]])
        specs.append(sp)
        del h, psd, noise
    return events, pools, specs, cuts


def run_stream(srv, ids, pools, n, rate, precision, seed=5999):
    """Submit n requests at Poisson arrival times; latency = done - arrival (host clock)."""
    import queue
    import threading
    from paper_2404_11397_amd import clock_ns
    offs, evs, pidx = synth.serving_stream(n, rate, seed=seed)
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
            "admit_wait_p99_ms": float(np.percentile(wait_adm, 99)),
            "service_p50_ms": float(np.percentile(lat - wait_adm, 50)),
            "service_p99_ms": float(np.percentile(lat - wait_adm, 99)), "evals_per_s": float(chains.sum() / span),
            "offered_evals_per_s": float(chains.sum() / (offs[-1] + 1e-9))}


def run_burst(srv, ids, pools, n, precision, seed=6001):
    """Submit n requests at once (the serving stream's events and batches, all arriving
    together) and wait for all: the server's capacity when it has a backlog."""
    from paper_2404_11397_amd import clock_ns
    _, evs, pidx = synth.serving_stream(n, synth.SERVE_RATE_HZ, seed=seed)
    before = srv.stats()
    t0 = clock_ns()
    tickets = [srv.submit(ids[e], pools[e][k], precision=precision, grad=True, t_arrival_ns=t0)
               for e, k in zip(evs, pidx)]
    done = max(srv.wait(t)[2]["t_done_ns"] for t in tickets)
    after = srv.stats()
    chains = sum(pools[e][k].shape[0] for e, k in zip(evs, pidx))
    return {"requests": n, "chains": int(chains), "seconds": (done - t0) * 1e-9,
            "evals_per_s": chains / ((done - t0) * 1e-9),
            "merged_launches": after["merged_launches"] - before["merged_launches"],
            "merged_requests": after["merged_requests"] - before["merged_requests"]}


def serving(torch, n_requests):
    """The multi-event request stream: 64 resident events, Poisson arrivals, lnL+grad
    per request.  Served by the library's request server (mixed precision, 4 streams,
    graph replays, merged launches of queued requests of one event) and, for comparison, one
    FIFO with FP64 plain launches, one request per launch.  Beside the Poisson streams, a
    burst of all requests at once measures each server's capacity with a backlog."""
    from paper_2404_11397_amd import Server
    t_build = time.perf_counter()
    events, pools, specs, cuts = build_serving_events(torch)
    t_build = time.perf_counter() - t_build
    budget = 32 << 30
    res = {"workload": f"{synth.N_SERVE_EVENTS} resident events (1-3 det, 32-256 s, 100-1000 bins, TaylorF2 / "
                       f"IMRPhenomD_NRTidalv2, 256-4096 chains each); Poisson {synth.SERVE_RATE_HZ:.0f} req/s of "
                       "lnL+grad requests",
           "events_build_s": t_build, "hbm_budget_bytes": budget,
           "injections": "as configured (no parameter changed)",
           "nrtv2_events_with_band_cut": len(cuts),
           "nrtv2_band_cut": "untapered reference amplitude reaches zero in band: the band ends at the last grid "
                             "point of the tapered injection (below 1.2 f_merger); band ends [Hz]: "
                             + ", ".join(f"{k}: {v:.0f}" for k, v in sorted(cuts.items())),
           "nrtv2_parity_vs_published_model": NRTV2_NOTE}
    for tag, streams, graphs, spin, merge, prec in (("server", 4, True, True, True, "mixed"),
                                                    ("baseline_fifo_fp64_plain", 1, False, False, False, "fp64")):
        with Server(budget, n_streams=streams, graphs=graphs, spin=spin, merge=merge) as srv:
            ids = [srv.add_event(e) for e in events]
            # warm-up to the steady state: every (event, pool) once, one at a time, then a
            # short Poisson stream (the buffers a light load rotates through), each followed
            # by a pause in which the idle worker captures the graphs of the new keys
            for e in range(len(events)):
                for k in range(len(pools[e])):
                    srv.wait(srv.submit(ids[e], pools[e][k], precision=prec))
            time.sleep(1.0)
            run_stream(srv, ids, pools, n_requests // 2, 2 * synth.SERVE_RATE_HZ, prec, seed=77)
            time.sleep(1.0)
            r = run_stream(srv, ids, pools, n_requests, synth.SERVE_RATE_HZ, prec)
            r["saturation"] = [run_stream(srv, ids, pools, n_requests, rate, prec) for rate in (2000.0, 20000.0)]
            r["burst"] = run_burst(srv, ids, pools, n_requests, prec)
            r["stats"] = srv.stats()
            r["streams"], r["graphs"], r["spin"] = streams, graphs, spin
            res[tag] = r
    res["resident_bytes"] = res["server"]["stats"]["resident_bytes"]
    return res


def mala_rate(torch, ev, w, steps):
    """Device MALA local steps (proposal, lnL+grad, accept) on the headline event: chain-steps/s.

    Chains start around the injection with spreads sigma_i = 1/sqrt(-d2 lnL/dz_i2) there (the
    diagonal of the observed information), the step is s_i = (f sigma_i)^2, and f is adapted
    during the untimed warm-up towards an acceptance of about 0.6; the timed steps keep f fixed."""
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
    sigma = diag_information_sigma(lambda x: Mala(ev, torch.as_tensor(x, device="cuda:0")).gz.cpu().numpy(),
                                   z0, hi - lo, 0.05 * (hi - lo))
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
    # a fresh set of random numbers for every step (timed, stamped and acceptance steps), drawn
    # before the timed region: reused sets would replay a rejected proposal until a chain sticks
    n_rand = 2 * steps + KERNEL_PASS_CALLS + 8
    xi = torch.randn((n_rand, B, 13), dtype=torch.float64, device="cuda:0", generator=gen)
    logu = torch.log(torch.rand((n_rand, B), dtype=torch.float64, device="cuda:0", generator=gen))
    xis, logus = list(xi), list(logu)
    k = [0]

    def one():
        ch.step(step, lo, hi, xis[k[0] % n_rand], logus[k[0] % n_rand])
        k[0] += 1

    # the clock ramp runs lnL+grad calls on the same event and batch size: the chains advance
    # only by the warm-up, timed and acceptance steps
    th_r = torch.as_tensor(w["theta"], device="cuda:0")
    out_r = (torch.empty(B, dtype=torch.float64, device="cuda:0"),
             torch.empty((B, 13), dtype=torch.float64, device="cuda:0"))
    ws_r = ev.workspace(B, with_grad=True)
    el, ku, su = time_calls(torch, one, steps, 2,
                            ramp_fn=lambda: ev.loglike_grad(th_r, out=out_r, workspace=ws_r))
    acc = torch.zeros(B, dtype=torch.int64, device="cuda:0")  # acceptance, outside the timed region
    for j in range(steps):
        acc += ch.step(step, lo, hi, xis[k[0] % n_rand], logus[k[0] % n_rand])
        k[0] += 1
    return {"chain_steps_per_s": B * steps / el, "us_per_step": el / steps * 1e6, "kernel_us": ku, "setup_us": su,
            "chains": B, "steps": steps, "acceptance": float(acc.sum()) / (B * steps), "step_factor": f,
            "precision": "fp64",
            "what": "rbl_mala_step on the headline event: two kernels, the gradient setup with the Langevin "
                    "proposal in its prologue and the lnL+grad kernel with the Metropolis decision in its "
                    "epilogue; chains around the injection, preconditioned by the diagonal observed information, "
                    "step adapted in warm-up; a fresh pre-drawn set of random numbers for every step"}


def progress(msg):
    """One line per finished section on stderr (stdout carries only the JSON result)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the likelihood shards over "
                                   "chains with no exchange, so no multi-GPU figure is measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    workload = "tf2_3det_128s_grad8192"
    cpu = None if args.no_cpu_baseline else cpu_baseline(workload, args.cpu_seconds)
    progress("oracle CPU baseline done")
    import torch

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
    ramp_calls, ramp_s = LAST_RAMP["calls"], LAST_RAMP["seconds"]
    progress(f"headline done: {B * args.steps / elapsed:.4g} evals/s")

    # per-call latency of a synchronised batch call
    lat = []
    for _ in range(50):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)

    forms = forms_on(torch, ev, theta, lnl, grad, ws, max(20, args.steps // 4), n_nodes=w["n_bins"] + 1,
                     n_det=len(w["tensors"]))

    nd = len(w["tensors"])
    psd = torch.as_tensor(w["psd"], device="cuda:0")
    summ_us = summary_pass(torch, w, edges, data, psd, ramp_fn=step)
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
        "clock_ramp": {"untimed_calls": ramp_calls, "seconds": ramp_s,
                       "what": f"untimed calls before the timed region: steps until {CLOCK_RAMP_S} s of "
                               f"back-to-back work had passed (the GPU raises its clocks over the first ~30 ms "
                               f"of sustained work), then the {args.warmup} warm-up steps"},
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
                     "kernel_timing": f"HIP start/stop events recorded by the runtime at the kernel's own start "
                                      f"and end on its launch stream, in a separate pass of "
                                      f"{min(args.steps, KERNEL_PASS_CALLS)} calls after the timed region",
                     "kernel_source_hash": kernel_source_hash()},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one synchronised rbl_loglike_grad call over the 8192-chain batch"},
        "forms": forms,
        "summary_pass": {"us": summ_us, "bytes": summ_bytes, "GB_per_s": summ_bytes / (summ_us * 1e-6) / 1e9,
                         "frac_of_hbm_peak": summ_bytes / (summ_us * 1e-6) / 1e9 / PEAK_HBM_GBS},
    }
    progress("forms and summary pass done")
    out["mala"] = mala_rate(torch, ev, w, max(20, args.steps))
    progress("MALA done")
    out["full_band"] = full_band(torch, max(10, args.steps // 10))
    out["reference_search"] = reference_search(torch)
    progress("reference search done")
    tr = stored_traffic("k_loglike_grad_tf2_3det_128s_8192_fp64")
    if tr is not None:
        out["roofline"]["traffic"] = tr["hbm_bytes_per_launch"]
        out["roofline"]["traffic_detail"] = tr
    if not args.no_nrtv2:
        out["nrtv2"] = nrtv2_forms(torch, max(20, args.steps // 4))
        progress("IMRPhenomD_NRTidalv2 forms done")
    if not args.no_serve:
        sv = serving(torch, args.serve_requests)
        progress("serving done")
        out["serving"] = sv
        out["latency_ms"] = {"p50": sv["server"]["p50_ms"], "p99": sv["server"]["p99_ms"],
                             "what": "request latency (arrival to results in host memory) under the "
                                     "multi-event Poisson stream, request server",
                             "batch_call_p50": float(np.percentile(lat, 50)),
                             "batch_call_p99": float(np.percentile(lat, 99))}
    if args.calibrate_copy:
        out["copy_calibration"] = calibrate_copy(torch)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
