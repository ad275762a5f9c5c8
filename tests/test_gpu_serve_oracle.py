"""Served results against the oracle: serving events with their configured injections
(1-3 detectors, both waveforms, 107-994 bins, 32-256 s), whole request batches through
the request server in FP64 and mixed precision with the gradient, checked on sampled
chains against the FP64 oracle (lnL: 1e-8 of the condition scale for FP64, 1e-2
absolute for mixed; gradient: 1e-5 of the largest prior-width-scaled component)."""
import numpy as np
import pytest

from gpu_common import WIDTHS, gpu_event, rb_condition_scale, say, serving_oracle_event
from oracle import likelihood as L

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

# (event id: waveform, detectors, duration, bins)  15: TaylorF2 3 det 64 s 107; 46: TaylorF2 2 det
# 32 s 938; 47: TaylorF2 1 det 32 s 884; 49: NRTidalv2 3 det 32 s 773; 0: NRTidalv2 2 det 32 s 533
# (band cut); 42: NRTidalv2 1 det 32 s 149 (band cut); 59: NRTidalv2 3 det 256 s 994 (band cut);
# 52: NRTidalv2 3 det 256 s 149
EVENTS = (15, 46, 47, 49, 0, 42, 59, 52)
N_SAMPLE = 10


@pytest.fixture(scope="module")
def served():
    out = []
    for eid in EVENTS:
        ev, sp, pool, cut = serving_oracle_event(eid)
        say(f"serving event {eid}: {sp['waveform']} D={sp['n_det']} T={sp['duration']:.0f} s bins={sp['n_bins']} "
            f"B={sp['batch']} band end {'%.1f Hz' % cut if cut else '2048 Hz'}")
        out.append((eid, ev, gpu_event(ev), pool[0], cut))
    return out


def test_served_lnl_and_grad_match_oracle(served):
    from paper_2404_11397_amd import Server
    assert any(c is not None for *_, c in served), "no event with a band cut"
    with Server(8 << 30, n_streams=4, graphs=True, spin=True) as srv:
        tickets = []
        for eid, ev, gev, th, _ in served:
            sid = srv.add_event(gev)
            for prec in ("fp64", "mixed"):
                tickets.append((srv.submit(sid, th, precision=prec, grad=True), eid, ev, th, prec))
        rng = np.random.default_rng(123)
        for t, eid, ev, th, prec in tickets:
            lnl, grad, _ = srv.wait(t)
            B = th.shape[0]
            idx = np.unique(np.concatenate([[0, B - 1], rng.choice(B, N_SAMPLE, replace=False)]))
            want_l, want_g = L.loglike_rb_grad(ev, th[idx])
            got_l, got_g = lnl[idx], grad[idx]
            if prec == "fp64":
                scale = np.maximum(np.abs(want_l), rb_condition_scale(ev, th[idx]))
                err_l = float(np.max(np.abs(got_l - want_l) / scale))
                gs, ws = got_g * WIDTHS, want_g * WIDTHS
                err_g = float(np.max(np.abs(gs - ws).max(axis=1) / np.abs(ws).max(axis=1)))
                say(f"  event {eid} fp64: lnL scaled err {err_l:.2e}, grad rel err {err_g:.2e}")
                assert err_l <= 1e-8, eid
                assert err_g <= 1e-5, eid
            else:
                err_l = float(np.max(np.abs(got_l - want_l)))
                say(f"  event {eid} mixed: lnL abs err {err_l:.2e}")
                assert err_l <= 1e-2, eid
