"""The Eq. (6) mismatch helper of the waveform-accuracy test, on known cases (no GPU)."""
import numpy as np

import synth
from _mismatch import mismatch


def test_pure_time_and_phase_shift_has_zero_mismatch():
    f_low, df, n, f = synth.frequency_grid(20.0, 2048.0, 128.0)
    psd = synth.analytic_psd(f)
    h1 = f ** (-7 / 6) * np.exp(-1j * (f / 3.0) ** 1.3)
    for dt, dphi in ((0.25, 0.7), (-1.5, 2.0), (0.0, -0.3)):
        h2 = h1 * np.exp(-2j * np.pi * f * dt + 1j * dphi)
        assert abs(mismatch(h1, h2, psd, f_low, df)) < 1e-12


def test_known_loss():
    """h2 = sqrt(1 - eps) h1 + sqrt(eps) g with g orthogonal to h1 at every shift probed except
    its own: the best shift keeps the h1 part, M = 1 - sqrt(1 - eps) up to the small overlap."""
    f_low, df, n, f = synth.frequency_grid(20.0, 512.0, 16.0)
    psd = synth.analytic_psd(f)
    rng = np.random.default_rng(5)
    h1 = f ** (-7 / 6) * np.exp(-1j * (f / 3.0) ** 1.3)
    g = f ** (-7 / 6) * np.exp(2j * np.pi * rng.uniform(size=n))    # random phases: ~orthogonal
    g *= np.sqrt(np.sum(np.abs(h1) ** 2 / psd) / np.sum(np.abs(g) ** 2 / psd))
    for eps in (1e-2, 1e-4):
        h2 = np.sqrt(1 - eps) * h1 + np.sqrt(eps) * g
        m = mismatch(h1, h2, psd, f_low, df)
        want = 1 - np.sqrt(1 - eps) / np.sqrt(1.0)   # <h2, h2> = <h1, h1> up to the cross term
        assert abs(m - want) < 0.2 * want, (eps, m, want)
