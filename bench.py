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

# Peaks of one MI355X (vendor figures): FP64 vector 78.6 TFLOP/s, HBM 8 TB/s.
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def flops_per_eval(n_nodes, n_det, grad, waveform="taylorf2"):
    """Counted algorithmic FP64 flops of one chain's relative-binned lnL (+ gradient).

    Counting FMA = 2, add/mul = 1, and each sin/cos pair of a phase in revolutions at
    its minimal polynomial cost (exact reduction 2 + 17 FMA = 36).  Per edge: TaylorF2
    phase in the separable basis (8 mul + 10 FMA = 28); per edge and detector: phase
    with delay (2), sin/cos (36), ratio K u (6), the binned terms and their sums (14).
    The gradient adds per edge and detector the edge adjoint and its accumulations (26)
    and per edge the basis accumulations (20).  Per chain: setup 600 (lnL) or 6000
    (with the 13-tangent Jacobian).
    """
    per_node = 28 + n_det * (2 + 36 + 6 + 14)
    setup = 600
    if grad:
        per_node += n_det * 26 + 20
        setup = 6000
    return n_nodes * per_node + setup


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def build_event(torch, workload):
    import synth
    from paper_2404_11397_amd import Event, bin_edges, strain
    w = synth.workload(workload)
    dev = torch.device("cuda:0")
    edges = bin_edges(w["f_low"], w["delta_f"], w["n_freq"], w["n_bins"])
    th0 = w["theta_inj"]
    h = strain(w["waveform"], w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"],
               w["n_freq"], th0, device=dev)
    data = h + torch.as_tensor(w["noise"], device=dev)
    psd = torch.as_tensor(w["psd"], device=dev)
    ev = Event(data, psd, w["tensors"], w["vertices"], w["gmst"], w["f_low"], w["delta_f"], th0, edges,
               waveform=w["waveform"], device=dev)
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


def time_calls(torch, fn, steps, warmup):
    """Wall time per call and HIP-event kernel times (main, setup) per call."""
    from paper_2404_11397_amd import profile_enable, profile_read
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    main_ms, setup_ms, calls = profile_read()
    profile_enable(False)
    return elapsed, main_ms / calls * 1e3, setup_ms / calls * 1e3


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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the likelihood shards over "
                                   "chains with no exchange, so no multi-GPU figure is measured",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    workload = "cfg4_tf2"
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

    # the other forms on the same batch (context beside the headline)
    forms = {}
    k = max(20, args.steps // 4)
    for name, prec, g in (("lnl_fp64", "fp64", False), ("lnl_mixed", "mixed", False),
                          ("lnl_grad_fp64", "fp64", True), ("lnl_grad_mixed", "mixed", True)):
        if g:
            fn = lambda p=prec: ev.loglike_grad(theta, p, out=(lnl, grad), workspace=ws)  # noqa: E731
        else:
            fn = lambda p=prec: ev.loglike(theta, p, out=lnl, workspace=ws)  # noqa: E731
        el, ku, su = time_calls(torch, fn, k, 3)
        forms[name] = {"evals_per_s": B * k / el, "us_per_call": el / k * 1e6, "kernel_us": ku, "setup_us": su}

    nd = len(w["tensors"])
    psd = torch.as_tensor(w["psd"], device="cuda:0")
    summ_us = summary_pass(torch, w, edges, data, psd)
    summ_bytes = w["n_freq"] * nd * 24  # data (complex128) + PSD (float64) per grid point and detector

    n_nodes = w["n_bins"] + 1
    fl = flops_per_eval(n_nodes, nd, grad=True)
    fl_kernel = fl - 6000
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
        "data": "synthetic (library TaylorF2 injection + seeded Gaussian noise, analytic PSD)",
        "config": {"workload": "TaylorF2 lnL+grad: 3 det, 128 s, 20-2048 Hz (259585 pts/det), "
                               "500 bins, 8192 chains, GW170817 prior",
                   "global_batch": B, "n_bins": w["n_bins"], "n_det": nd, "n_freq": w["n_freq"],
                   "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_loglike_grad<3>", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": None, "flops_per_eval": fl_kernel,
                     "avg_kernel_us": kern_us, "avg_setup_us": setup_us},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one synchronised rbl_loglike_grad call over the 8192-chain batch"},
        "forms": forms,
        "summary_pass": {"us": summ_us, "bytes": summ_bytes, "GB_per_s": summ_bytes / (summ_us * 1e-6) / 1e9,
                         "frac_of_hbm_peak": summ_bytes / (summ_us * 1e-6) / 1e9 / PEAK_HBM_GBS},
    }
    if not args.no_cpu_baseline:
        data_host = data.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(w, edges, data_host, theta_np, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
