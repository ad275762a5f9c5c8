"""Full-band likelihood (Eqs. (2)-(3) on every grid point, rbl_loglike_full) at the
workload grid sizes: the 3-detector 128 s TaylorF2 grid (259585 points per detector) and
the 3-detector 256 s IMRPhenomD_NRTidalv2 grid (519169 points), against the oracle on
sampled chains (1e-8 of max(|lnL|, <h, h>)); a ragged batch with invalid chains; bitwise
repeatability."""
import numpy as np
import pytest

from gpu_common import gpu_event, oracle_event, say
from oracle import likelihood as L

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _cuda(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name,B,n_sample", [("tf2_3det_128s", 4096, 6), ("nrtv2_3det_256s", 1001, 3)])
def test_full_band_parity_at_workload_size(name, B, n_sample):
    ev, w = oracle_event(name, batch=B)
    gev = gpu_event(ev, keep_grid=True)
    th = w["theta"]
    t = _cuda(th)
    got = gev.loglike_full(t).cpu().numpy()
    again = gev.loglike_full(t).cpu().numpy()
    assert np.array_equal(got, again)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([[0, B - 1], rng.choice(B, n_sample, replace=False)]))
    want = L.loglike_full(ev, th[idx])
    hh = L.optimal_snr2(ev, th[idx])
    err = np.abs(got[idx] - want) / np.maximum(np.abs(want), hh)
    say(f"{name} full band, {B} chains: max scaled err {err.max():.2e} over {len(idx)} sampled chains")
    assert np.all(err <= 1e-8)
    # the binned lnL at the reference equals the full one
    th0 = w["theta_inj"][None, :]
    rb = gev.loglike(_cuda(th0)).cpu().numpy()[0]
    full0 = gev.loglike_full(_cuda(th0)).cpu().numpy()[0]
    if name.startswith("tf2"):
        assert rb == pytest.approx(full0, rel=1e-11)


def test_full_band_ragged_batch_with_invalid_chains():
    ev, w = oracle_event("tf2_1det_32s", batch=13)
    gev = gpu_event(ev, keep_grid=True)
    th = w["theta"].copy()
    th[3, 0] = np.nan       # NaN -> NaN
    th[5, 6] = -10.0        # outside the domain -> -inf
    th[11, 2] = 1.5
    got = gev.loglike_full(_cuda(th)).cpu().numpy()
    assert np.isnan(got[3]) and got[5] == -np.inf and got[11] == -np.inf
    ok = [i for i in range(13) if i not in (3, 5, 11)]
    want = L.loglike_full(ev, th[ok])
    hh = L.optimal_snr2(ev, th[ok])
    assert np.all(np.abs(got[ok] - want) / np.maximum(np.abs(want), hh) <= 1e-8)
