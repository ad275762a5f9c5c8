"""Detector response: antenna patterns and geocentre time delay.

The paper projects the two polarisations onto each interferometer of the
network (Sec. II A, through its parameter list in Tab. II: polarisation angle,
right ascension, declination).  Conventions (the paper is silent):
  * source direction n = (cos dec cos phi, cos dec sin phi, sin dec),
    phi = ra - gmst, in the Earth-fixed frame; no Earth rotation over a segment;
  * polarisation axes p = cos(psi) e_theta + sin(psi) e_phi,
    q = sin(psi) e_theta - cos(psi) e_phi, with e_theta, e_phi the polar and
    azimuthal unit vectors at the source direction;
  * e_plus = p p^T - q q^T, e_cross = p q^T + q p^T, F = D : e;
  * arrival delay relative to the geocentre dt = -(r . n) / c.
For a detector with arms along x and y these reproduce the textbook
F+ = (1+cos^2 th)/2 cos 2ph cos 2psi - cos th sin 2ph sin 2psi and
Fx = (1+cos^2 th)/2 cos 2ph sin 2psi + cos th sin 2ph cos 2psi
(pinned in the tests).
"""
import numpy as np

from . import ad
from .constants import C_SI


def _unit_vectors(ra, dec, gmst):
    phi = ra - gmst
    cp, sp = ad.cos(phi), ad.sin(phi)
    cd, sd = ad.cos(dec), ad.sin(dec)
    n = (cd * cp, cd * sp, sd)
    e_th = (sd * cp, sd * sp, -1.0 * cd)
    e_ph = (-1.0 * sp, cp, 0.0 * cp)
    return n, e_th, e_ph


def antenna_patterns(tensor, ra, dec, psi, gmst):
    """(F+, Fx) for one detector tensor [3, 3]; angles broadcast."""
    _, e_th, e_ph = _unit_vectors(ra, dec, gmst)
    c, s = ad.cos(psi), ad.sin(psi)
    p = [c * e_th[i] + s * e_ph[i] for i in range(3)]
    q = [s * e_th[i] - c * e_ph[i] for i in range(3)]
    fp = 0.0
    fc = 0.0
    for i in range(3):
        for j in range(3):
            dij = float(tensor[i][j])
            if dij == 0.0:
                continue
            fp = fp + dij * (p[i] * p[j] - q[i] * q[j])
            fc = fc + dij * (p[i] * q[j] + q[i] * p[j])
    return fp, fc


def time_delay(vertex, ra, dec, gmst):
    """Arrival time at the detector minus arrival time at the geocentre [s]."""
    n, _, _ = _unit_vectors(ra, dec, gmst)
    dot = 0.0
    for i in range(3):
        dot = dot + float(vertex[i]) * n[i]
    return -1.0 * dot / C_SI
