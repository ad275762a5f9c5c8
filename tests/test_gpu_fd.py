"""Gradient of the library against central finite differences of its own FP64 lnL
(h = 1e-6 relative, as the differentiation workload specifies), for both waveforms.
Angles and t_c take an absolute step; the comparison is per chain with components
scaled by the prior widths."""
import numpy as np
import pytest

from _events import near_draws
from gpu_common import WIDTHS, gpu_event, oracle_event, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", ["tf2_3det_128s", "nrtv2_3det_256s"])
def test_gradient_matches_central_differences(name):
    ev, _ = oracle_event(name, batch=8)
    gev = gpu_event(ev)
    th = near_draws(ev.theta_ref, 8, 50, scale=0.3)
    _, g = gev.loglike_grad(_cuda(th))
    g = g.cpu().numpy()
    step = 1e-6 * np.maximum(np.abs(th), 1.0)
    rows = []
    for i in range(13):
        tp, tm = th.copy(), th.copy()
        tp[:, i] += step[:, i]
        tm[:, i] -= step[:, i]
        rows.append((tp, tm))
    allp = np.concatenate([r[0] for r in rows] + [r[1] for r in rows])
    vals = gev.loglike(_cuda(allp)).cpu().numpy().reshape(2, 13, len(th))
    fd = ((vals[0] - vals[1]) / (2 * step.T)).T
    gs, fs = g * WIDTHS, fd * WIDTHS
    rel = np.abs(gs - fs).max(axis=1) / np.abs(gs).max(axis=1)
    say(name, "adjoint vs central differences, max rel err", rel.max())
    assert np.all(rel <= 1e-4)
