"""Host logic of the benchmark: the clock ramp before every timed region, and the committed
HBM-traffic summary, which the benchmark reports only while it matches the kernel sources."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _FakeCuda:
    def __init__(self):
        self.syncs = 0

    def synchronize(self):
        self.syncs += 1


class _FakeTorch:
    def __init__(self):
        self.cuda = _FakeCuda()


def test_ramp_runs_for_its_duration_then_the_warmup_calls():
    torch = _FakeTorch()
    order = []
    n, dt = bench.ramp(torch, lambda: order.append("step"), 5, ramp_fn=lambda: order.append("ramp"),
                       seconds=0.02)
    assert dt >= 0.02
    assert order[-5:] == ["step"] * 5            # the warm-up calls come last, back to back
    assert set(order[:-5]) == {"ramp"} and len(order) == n
    assert torch.cuda.syncs >= (n - 5) // 16      # the host waits for the device every 16 calls


def test_ramp_without_a_ramp_function_uses_the_timed_call():
    torch = _FakeTorch()
    calls = []
    t0 = time.perf_counter()
    n, _ = bench.ramp(torch, lambda: calls.append(1), 3, seconds=0.01)
    assert time.perf_counter() - t0 >= 0.01
    assert len(calls) == n and n >= 3


def test_committed_traffic_summary_matches_the_kernel_sources():
    rec = bench.stored_traffic("k_loglike_grad_tf2_3det_128s_8192_fp64")
    assert rec is not None, "profiles/..._traffic.md was taken on other kernel sources: profile again"
    assert rec["source_hash"] == bench.kernel_source_hash()
    assert 0.9 < rec["read_scale"] / 2.0 < 1.1 and 0.9 < rec["write_scale"] < 1.1
    assert rec["hbm_bytes_per_launch"] > 8192 * 216   # at least theta in, lnL and gradient out
