"""Waveform accuracy as the paper measures it (Sec. III A, Eq. (6)): the mismatch
M = 1 - max over (dt_c, dphi_c) of <h1, h2> / sqrt(<h1, h1> <h2, h2>) between the library's
strain (rbl_strain, on the device) and the oracle's strain, for both waveforms (the
IMRPhenomD_NRTidalv2 stand-in with its Planck taper), over draws from the paper's Tab. I
ranges, on the grid [20, 2048] Hz with df = 1/T, T = 128 s, with the analytic PSD standing
in for the design-sensitivity curve.  The maximum over the time shift is taken from an
inverse FFT of the noise-weighted cross spectrum, the maximum over the phase by its modulus.
The paper samples 10000 draws per model; this test takes 100 per waveform."""
import numpy as np
import pytest

import synth
from _mismatch import mismatch
from gpu_common import say
from oracle import waveform as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

N_DRAWS = 100


@pytest.mark.parametrize("waveform", ["taylorf2", "phenomd_nrtv2"])
def test_library_vs_oracle_mismatch(waveform):
    from paper_2404_11397_amd import strain
    f_low, df, n, f = synth.frequency_grid(20.0, 2048.0, 128.0)
    psd = synth.analytic_psd(f)
    tensor, vertex = synth.detector_geometry(0.0, 0.0, 0.0)
    th = synth.mismatch_draws(6000 + (waveform == "phenomd_nrtv2"), N_DRAWS)
    ms = []
    for t in th:
        hg = strain(waveform, tensor[None], vertex[None], 0.0, f_low, df, n, t, taper=True)[0].cpu().numpy()
        ho = W.strain(f, t, tensor[None], vertex[None], 0.0, waveform, True)[0][0]
        ms.append(mismatch(hg, ho, psd, f_low, df))
    ms = np.array(ms)
    say(f"{waveform}: mismatch over {N_DRAWS} Tab. I draws: max {ms.max():.2e}, median {np.median(ms):.2e}, "
        f"min {ms.min():.2e}")
    assert np.all(np.abs(ms) < 1e-12)
