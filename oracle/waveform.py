"""Projected frequency-domain strain of one binary in each detector.

  h_d(f) = (C_d / dL) A(f) exp(-i Psi_int(f)) exp(2 i phic) exp(-2 pi i f (tc + dt_d))
  C_d    = (1 + cos^2 iota)/2 F+_d - i cos(iota) Fx_d

i.e. h_plus = (1+cos^2 iota)/2 H, h_cross = -i cos(iota) H with the core
waveform H = A exp(-i Psi), Psi = 2 pi f tc - 2 phic + Psi_int, the sign of the
exponent following the ratio of Eq. (4).  phic is the orbital coalescence phase
(the dominant mode carries twice it).  Parameters enter as arrays broadcasting
against f (shape [B, 1] against [N]) or as Duals for gradients.
"""
import numpy as np

from . import ad, detector, taylorf2

TWO_PI = 2.0 * np.pi


def unpack(theta):
    """theta [B, 13] (array or list of 13 Duals) -> list of 13 column views [B, 1]."""
    if isinstance(theta, (list, tuple)):
        return list(theta)
    theta = np.asarray(theta, dtype=np.float64)
    if theta.ndim == 1:
        theta = theta[None, :]
    return [theta[:, i:i + 1] for i in range(13)]


def intrinsic(f, p, approximant, taper=True):
    """(amplitude at 1 Mpc, Psi_int) for the intrinsic parameters p[0:6]."""
    mc, q, chi1, chi2, l1, l2 = p[:6]
    if approximant == "taylorf2":
        return taylorf2.amplitude(f, mc), taylorf2.phase(f, mc, q, chi1, chi2, l1, l2)
    if approximant == "phenomd_nrtv2":
        from . import phenomd_nrtv2
        return phenomd_nrtv2.amplitude_phase(f, mc, q, chi1, chi2, l1, l2, taper=taper)
    raise ValueError(f"unknown approximant {approximant!r}")


def projection(p, tensors, vertices, gmst):
    """Per detector: complex response C_d and time delay dt_d (lists over d)."""
    iota, psi, ra, dec = p[9], p[10], p[11], p[12]
    ci = ad.cos(iota)
    out = []
    for tensor, vertex in zip(tensors, vertices):
        fp, fc = detector.antenna_patterns(tensor, ra, dec, psi, gmst)
        c_d = 0.5 * (1.0 + ci * ci) * fp - 1j * (ci * fc)
        dt = detector.time_delay(vertex, ra, dec, gmst)
        out.append((c_d, dt))
    return out


def strain(f, theta, tensors, vertices, gmst, approximant, taper=True):
    """Projected strain h_d(f; theta) -> list over detectors of [B, len(f)]."""
    p = unpack(theta)
    amp, psi_int = intrinsic(f, p, approximant, taper)
    dl, tc, phic = p[6], p[7], p[8]
    core = amp * ad.exp(-1j * psi_int + 2j * phic) / dl
    out = []
    for c_d, dt in projection(p, tensors, vertices, gmst):
        out.append(c_d * core * ad.exp(-1j * TWO_PI * f * (tc + dt)))
    return out
