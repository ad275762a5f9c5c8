"""Reference-parameter search (Sec. II C) through the C-ABI: rbl_ref_search (CMA-ES on the
device full-band lnL) follows the oracle's CMA-ES generation by generation when both get the
same normals (fitness from the GPU and from the oracle differ only by rounding, so the
rankings agree)."""
import numpy as np
import pytest

from gpu_common import gpu_event, say
from oracle import cmaes
from oracle import likelihood as L

from _events import small_event

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def test_ref_search_follows_the_oracle_cmaes():
    from paper_2404_11397_amd import ref_search
    ev = small_event(approximant="taylorf2", n_det=2, duration=8.0, f_high=512.0, n_bins=40)
    L.prepare(ev)
    gev = gpu_event(ev, keep_grid=True)
    half = np.array([1e-3, 0.1, 0.02, 0.02, 200, 200, 10, 1e-3, 0.5, 0.2, 0.2, 0.1, 0.1])
    lo, hi = ev.theta_ref - half, ev.theta_ref + half
    start = ev.theta_ref + 0.3 * half * np.sin(np.arange(13))
    normals = np.random.default_rng(8).standard_normal((15, 16, 13))
    best, best_l, trace = ref_search(gev, lo, hi, start, 0.2, normals)
    ob, obl, otrace = cmaes.search(lambda th: L.loglike_full(ev, th), lo, hi, start, 0.2, 16, normals)
    scale = np.abs(otrace[:, 0]).max()
    say(f"ref search vs oracle: best lnL {best_l:.6f} / {obl:.6f}; max mean diff (box units) "
        f"{np.max(np.abs(trace[:, 2:] - otrace[:, 2:]) / (hi - lo)):.2e}")
    np.testing.assert_allclose(trace[:, 0], otrace[:, 0], rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(trace[:, 1], otrace[:, 1], rtol=1e-9)
    assert np.max(np.abs(trace[:, 2:] - otrace[:, 2:]) / (hi - lo)) < 1e-9
    np.testing.assert_allclose(best, ob, rtol=0, atol=1e-9 * np.max(hi - lo))
