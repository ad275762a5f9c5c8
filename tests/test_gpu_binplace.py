"""Bin placement on the device (an event created without edges): the edges equal the
oracle's post-Newtonian phase-bound placement index for index on the workload grids and on
small and odd ones, and the event then gives the same likelihood as one created with those
edges."""
import numpy as np
import pytest

import synth
from gpu_common import say
from oracle import binning

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

CASES = [(20.0, 1024.0, 32.0, 100), (20.0, 2048.0, 128.0, 500), (20.0, 2048.0, 256.0, 1000),
         (20.0, 2048.0, 64.0, 777), (20.0, 30.0, 1.0, 10), (20.0, 300.0, 2.0, 559)]


@pytest.mark.parametrize("f_low,f_high,duration,n_bins", CASES)
def test_device_bin_placement_matches_oracle(f_low, f_high, duration, n_bins):
    from paper_2404_11397_amd import Event
    fl, df, n, f = synth.frequency_grid(f_low, f_high, duration)
    psd = synth.analytic_psd(f)[None, :]
    tensor, vertex = synth.detector_geometry(0.2, 0.3, 0.4)
    th0 = np.array([1.2, 0.8, 0.01, 0.0, 100.0, 200.0, 50.0, 0.0, 0.1, 0.4, 0.3, 1.0, 0.2])
    data = (synth.gaussian_noise(3, psd, duration)).astype(complex)
    dev = Event(data, psd, tensor[None], vertex[None], 0.3, fl, df, th0, n_bins)
    want = binning.pn_bin_edges(fl, df, n, n_bins)
    got = dev.edges()
    say(f"grid {n} points, {n_bins} bins: device edges equal the oracle's: {np.array_equal(got, want)}")
    assert np.array_equal(got, want)
    host = Event(data, psd, tensor[None], vertex[None], 0.3, fl, df, th0, want)
    th = torch.as_tensor(np.tile(th0, (5, 1)) + 1e-4 * np.arange(5)[:, None], device="cuda")
    assert torch.equal(dev.loglike(th), host.loglike(th))
