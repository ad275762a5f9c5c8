"""Request server on the GPU: every request's result is bitwise the same served alone
(a direct library call), in a concurrent mix and in a launch merged with other requests of
its event; admission by HBM footprint queues requests that do not fit and rejects those
that never can."""
import time

import numpy as np
import pytest

from gpu_common import gpu_event, oracle_event, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


@pytest.fixture(scope="module")
def events():
    specs = [("tf2_1det_32s", 300, 16.0, 100), ("tf2_3det_128s", 700, 16.0, 200), ("nrtv2_3det_256s", 1100, 16.0, 300), ("tf2_3det_128s", 256, 8.0, 120)]
    out = []
    for name, batch, dur, nb in specs:
        ev, w = oracle_event(name, batch=batch, duration=dur, n_bins=nb)
        out.append((gpu_event(ev), w["theta"]))
        say("event", name, "B", batch, "bins", nb)
    return out


def _alone(gev, th, precision, grad):
    t = torch.as_tensor(th, dtype=torch.float64, device="cuda")
    if grad:
        lnl, g = gev.loglike_grad(t, precision)
        return lnl.cpu().numpy(), g.cpu().numpy()
    return gev.loglike(t, precision).cpu().numpy(), None


@pytest.mark.parametrize("graphs,spin", [(True, False), (False, False), (True, True)])
def test_alone_equals_mix(events, graphs, spin):
    from paper_2404_11397_amd import Server
    rng = np.random.default_rng(11)
    plan = [(int(rng.integers(len(events))), prec, grad)
            for prec in ("fp64", "mixed") for grad in (True, False) for _ in range(6)]
    rng.shuffle(plan)
    with Server(4 << 30, n_streams=4, graphs=graphs, spin=spin) as srv:
        ids = [srv.add_event(gev) for gev, _ in events]
        # two passes over the plan: graphs missing in the first are captured while the
        # worker is idle in between, and replayed in the second
        for rep in range(2):
            if rep:
                time.sleep(0.5)  # the idle worker captures the graphs of the first pass
            tickets = [(srv.submit(ids[e], events[e][1], precision=p, grad=g), e, p, g) for e, p, g in plan]
            for t, e, p, g in tickets:
                lnl, grad, info = srv.wait(t)
                want_l, want_g = _alone(events[e][0], events[e][1], p, g)
                assert np.array_equal(lnl, want_l, equal_nan=True), (e, p, g)
                if g:
                    assert np.array_equal(grad, want_g, equal_nan=True), (e, p, g)
                assert info["t_arrival_ns"] <= info["t_admit_ns"] <= info["t_done_ns"]
        st = srv.stats()
        say("stats", st)
        assert st["completed"] == 2 * len(plan) and st["in_flight"] == 0 and st["queued"] == 0
        assert st["max_in_flight"] > 1
        # a merged launch serves merged_requests / merged_launches requests at once
        served = st["graph_launches"] + st["plain_launches"] + st["merged_requests"] - st["merged_launches"]
        assert served == 2 * len(plan)
        if graphs:
            assert st["graphs"] > 0 and st["graph_launches"] > 0
        else:
            assert st["graph_launches"] == 0 and st["graphs"] == 0


@pytest.mark.parametrize("merge", [True, False])
def test_merged_launches_equal_alone(events, merge):
    """Requests queued behind a long one are taken into one launch per (event, precision,
    gradient flag), up to 8192 chains, and each gets bitwise the results of its own call."""
    from paper_2404_11397_amd import Server
    rng = np.random.default_rng(12)
    gev_n, th_n = events[2]  # IMRPhenomD_NRTidalv2, 1100 chains: keeps the stream busy
    cuts = [(1, 0), (17, 3), (64, 40), (100, 7), (256, 1), (3, 250), (700, 0), (33, 600)]
    with Server(4 << 30, n_streams=1, graphs=False, merge=merge) as srv:
        ids = [srv.add_event(gev) for gev, _ in events]
        plan = [(2, th_n, "fp64", True)] * 3
        for n, at in cuts:
            e = int(rng.integers(2))  # the two TaylorF2 events with 300 and 700 chains
            th = events[e][1]
            n = min(n, len(th) - at % len(th))
            plan.append((e, th[at % len(th):at % len(th) + n], str(rng.choice(["fp64", "mixed"])),
                         bool(rng.integers(2))))
        plan += [(1, events[1][1], "mixed", True)] * 14  # 9800 chains of one kind: over one launch's 8192
        tickets = [(srv.submit(ids[e], th, precision=p, grad=g), e, th, p, g) for e, th, p, g in plan]
        for t, e, th, p, g in tickets:
            lnl, grad, info = srv.wait(t)
            want_l, want_g = _alone(events[e][0], th, p, g)
            assert np.array_equal(lnl, want_l, equal_nan=True), (e, len(th), p, g)
            if g:
                assert np.array_equal(grad, want_g, equal_nan=True), (e, len(th), p, g)
        st = srv.stats()
        say("merge", merge, "stats", st)
        assert st["completed"] == len(plan)
        assert st["plain_launches"] + st["merged_requests"] - st["merged_launches"] == len(plan)
        if merge:
            assert st["merged_launches"] >= 2 and st["merged_requests"] >= 5
            assert st["plain_launches"] < len(plan)
        else:
            assert st["merged_launches"] == 0 and st["plain_launches"] == len(plan)


def test_small_budget_queues_and_rejects(events):
    from paper_2404_11397_amd import RblError, Server
    gev, th = events[2]                       # 1100 chains -> 2048-chain buffer class
    fp = gev.footprint_bytes()
    with Server(1 << 40, n_streams=1) as probe:
        eid = probe.add_event(gev)
        probe.wait(probe.submit(eid, th[:1], precision="fp64"))
        one = probe.stats()["buffer_bytes"]   # a 256-chain buffer
    budget = fp + 9 * one                     # room for one 2048-chain buffer (8x), not two
    with Server(budget, n_streams=4) as srv:
        eid = srv.add_event(gev)
        ts = [srv.submit(eid, th, precision="mixed") for _ in range(6)]
        want_l, want_g = _alone(gev, th, "mixed", True)
        for t in ts:
            lnl, grad, _ = srv.wait(t)
            assert np.array_equal(lnl, want_l, equal_nan=True) and np.array_equal(grad, want_g, equal_nan=True)
        st = srv.stats()
        say("small budget stats", st)
        assert st["max_in_flight"] == 1 and st["admission_waits"] >= 1
        assert st["resident_bytes"] + st["buffer_bytes"] <= budget
        big = np.repeat(th, 4, axis=0)        # 4400 chains -> 8192 class: never fits
        with pytest.raises(RblError):
            srv.submit(eid, big)
    with Server(fp + 1, n_streams=1) as tight:  # room for one resident event only
        tight.add_event(gev)
        with pytest.raises(RblError):
            tight.add_event(events[1][0])


def test_remove_event_and_empty_request(events):
    from paper_2404_11397_amd import RblError, Server
    gev, th = events[0]
    with Server(1 << 32, n_streams=2) as srv:
        eid = srv.add_event(gev)
        t = srv.submit(eid, th)
        with pytest.raises(RblError):
            srv.remove_event(eid)
        srv.wait(t)
        t0 = srv.submit(eid, th[:0])
        lnl, _, _ = srv.wait(t0)
        assert lnl.shape == (0,)
        srv.remove_event(eid)
        with pytest.raises(RblError):
            srv.submit(eid, th)
