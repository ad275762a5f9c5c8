"""Device MALA step against the oracle's (same z, same random numbers): state after init,
accept decisions (chains whose log u lies within 1e-6 of log alpha are not compared), and
the chain state after several steps."""
import numpy as np
import pytest

from oracle import likelihood as L
from oracle import mala as M

from _events import near_draws, small_event
from gpu_common import WIDTHS, gpu_event, rb_condition_scale, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

STEP = (0.1 * np.array([2e-5, 1e-2, 2e-3, 2e-3, 20.0, 20.0, 1.0, 2e-5, 0.05, 0.02, 0.02, 0.01, 0.01])) ** 2


def _cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _to_z(th):
    z = th.copy()
    z[:, 9] = np.cos(th[:, 9])
    z[:, 12] = np.sin(th[:, 12])
    return z


@pytest.mark.parametrize("approximant", ["taylorf2", "phenomd_nrtv2"])
def test_mala_steps_match_oracle(approximant):
    from paper_2404_11397_amd import Mala
    ev = small_event(approximant=approximant, duration=4.0, f_high=512.0, n_bins=40)
    L.prepare(ev)
    gev = gpu_event(ev)
    B = 96
    z = _to_z(near_draws(ev.theta_ref, B, 61, scale=0.2))
    lo, hi = M.prior_box("injection")
    ch = Mala(gev, _cuda(z))
    lnl_o, gz_o = M.loglike_grad_z(ev, z)
    lnl_g, gz_g = ch.lnl.cpu().numpy(), ch.gz.cpu().numpy()
    scale = np.maximum(np.abs(lnl_o), rb_condition_scale(ev, M.z_to_theta(z)))
    assert np.all(np.abs(lnl_g - lnl_o) <= 1e-8 * scale)
    wz = WIDTHS.copy()
    wz[9] = wz[12] = 2.0
    rel = np.abs((gz_g - gz_o) * wz).max(axis=1) / np.abs(gz_o * wz).max(axis=1)
    assert np.all(rel <= 1e-5)
    rng = np.random.default_rng(62)
    zo, lo_, go = z.copy(), lnl_o.copy(), gz_o.copy()
    live = np.ones(B, bool)  # chains whose history matched so far
    n_acc = 0
    for it in range(5):
        xi = rng.standard_normal((B, 13))
        logu = np.log(rng.uniform(size=B))
        acc_g = ch.step(STEP, lo, hi, _cuda(xi), _cuda(logu)).cpu().numpy().astype(bool)
        zo, lo_, go, acc_o, la = M.mala_step(ev, zo, lo_, go, STEP, xi, logu, lo, hi)
        near = np.abs(la - logu) < 1e-6
        live &= ~near
        assert np.array_equal(acc_g[live], acc_o[live]), it
        zg, lg, gg = ch.z.cpu().numpy(), ch.lnl.cpu().numpy(), ch.gz.cpu().numpy()
        # the drift (s/2) g carries the gradient difference (<= 1e-10 relative here) into z
        np.testing.assert_allclose(zg[live], zo[live], rtol=1e-9, atol=1e-12)
        sc = np.maximum(np.abs(lo_[live]), rb_condition_scale(ev, M.z_to_theta(zo[live])))
        assert np.all(np.abs(lg[live] - lo_[live]) <= 1e-8 * sc)
        n_acc += acc_o[live].sum()
    say(approximant, "MALA: chains compared", live.sum(), "of", B, "accepted over 5 steps", n_acc)
    assert live.sum() >= B - 2 and 0 < n_acc < 5 * B


def test_mala_argument_checks():
    from paper_2404_11397_amd import Mala, RblError
    ev = small_event(duration=4.0, f_high=256.0, n_bins=20)
    L.prepare(ev)
    gev = gpu_event(ev)
    z = _to_z(near_draws(ev.theta_ref, 4, 63))
    ch = Mala(gev, _cuda(z))
    lo, hi = M.prior_box("injection")
    xi, logu = _cuda(np.zeros((4, 13))), _cuda(np.zeros(4))
    with pytest.raises(RblError):
        ch.step(-STEP, lo, hi, xi, logu)
    with pytest.raises(RblError):
        ch.step(STEP, hi, lo, xi, logu)
    acc = ch.step(STEP, lo, hi, xi, _cuda(np.full(4, -np.inf))).cpu().numpy()  # log u = -inf: accept if inside
    assert acc.all()


def test_mala_steps_match_oracle_at_workload_size():
    """1024 chains on the 3-detector 128 s TaylorF2 workload (259585 points per detector,
    500 bins), three fused steps against the oracle's."""
    from paper_2404_11397_amd import Mala
    from gpu_common import oracle_event
    ev, w = oracle_event("tf2_3det_128s", batch=8)
    gev = gpu_event(ev)
    B = 1024
    z = _to_z(near_draws(ev.theta_ref, B, 71, scale=0.05))
    b = __import__("synth").PRIORS["gw170817"]
    lo = np.array([b["Mc"][0], b["q"][0], b["chi"][0], b["chi"][0], b["L"][0], b["L"][0], b["dL"][0], b["tc"][0],
                   0.0, -1.0, 0.0, 0.0, -1.0])
    hi = np.array([b["Mc"][1], b["q"][1], b["chi"][1], b["chi"][1], b["L"][1], b["L"][1], b["dL"][1], b["tc"][1],
                   2 * np.pi, 1.0, np.pi, 2 * np.pi, 1.0])
    z = np.clip(z, lo, hi)
    step = (0.3 * np.array([2e-6, 2e-3, 4e-4, 4e-4, 30.0, 30.0, 0.5, 2e-5, 0.02, 0.01, 0.01, 0.005, 0.005])) ** 2
    ch = Mala(gev, _cuda(z))
    lnl_o, gz_o = M.loglike_grad_z(ev, z)
    rng = np.random.default_rng(72)
    zo, lo_, go = z.copy(), lnl_o.copy(), gz_o.copy()
    live = np.ones(B, bool)
    n_acc = 0
    for it in range(3):
        xi = rng.standard_normal((B, 13))
        logu = np.log(rng.uniform(size=B))
        acc_g = ch.step(step, lo, hi, _cuda(xi), _cuda(logu)).cpu().numpy().astype(bool)
        zo, lo_, go, acc_o, la = M.mala_step(ev, zo, lo_, go, step, xi, logu, lo, hi)
        live &= ~(np.abs(la - logu) < 1e-6)
        assert np.array_equal(acc_g[live], acc_o[live]), it
        zg, lg = ch.z.cpu().numpy(), ch.lnl.cpu().numpy()
        np.testing.assert_allclose(zg[live], zo[live], rtol=1e-9, atol=1e-12)
        sc = np.maximum(np.abs(lo_[live]), rb_condition_scale(ev, M.z_to_theta(zo[live])))
        assert np.all(np.abs(lg[live] - lo_[live]) <= 1e-8 * sc)
        n_acc += acc_o[live].sum()
    say("tf2_3det_128s MALA, 1024 chains: compared", live.sum(), "accepted over 3 steps", n_acc)
    assert live.sum() >= B - 4 and 0 < n_acc < 3 * B
