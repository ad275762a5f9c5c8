"""The waveform mismatch of the paper's Eq. (6) (test infrastructure)."""
import numpy as np


def mismatch(h1, h2, psd, f_low, df):
    """M = 1 - max over (dt, dphi) of Re<h1, h2 exp(i(2 pi f dt + dphi))> / sqrt(<h1, h1> <h2, h2>)
    for two strains on the grid f_k = f_low + k df: the maximum over the phase is the modulus
    of the complex inner product, the maximum over the time shift is read off an inverse FFT
    of the noise-weighted cross spectrum (placed at its absolute frequency bins, zero-padded
    to twice the band's top bin, so the shifts are multiples of 1/(n_fft df))."""
    n_fft = 1 << int(np.ceil(np.log2(2 * (f_low / df + len(h1)))))
    x = np.zeros(n_fft, complex)
    k0 = int(round(f_low / df))
    x[k0:k0 + len(h1)] = h1 * np.conj(h2) / psd
    z = np.abs(np.fft.ifft(x)) * n_fft * 4.0 * df
    n1 = 4.0 * df * np.sum(np.abs(h1) ** 2 / psd)
    n2 = 4.0 * df * np.sum(np.abs(h2) ** 2 / psd)
    return 1.0 - z.max() / np.sqrt(n1 * n2)
