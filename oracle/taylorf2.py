"""TaylorF2: the post-Newtonian frequency-domain inspiral the paper uses
(Sec. II B), aligned spins and tidal terms.

h(f) = A(f) exp(-i Psi_int(f)) at unit distance and unit antenna response;
the extrinsic factors (distance, coalescence time and phase, projection) are
applied in oracle.waveform.

Phase (stationary-phase approximation), v = (pi M f)^(1/3), M in seconds:
  Psi_int = -pi/4 + 3/(128 eta v^5) [ sum_{k=0..7} (phi_k + phi_k^l ln v) v^k
                                      + phi_10 v^10 + phi_12 v^12 ]
  * point-particle coefficients to 3.5PN (Buonanno, Iyer, Ochsner, Pan &
    Sathyaprakash 2009, the TaylorF2 phase), with the 2.5PN term written as
    (1 + 3 ln(v / v_lso)), v_lso = 6^(-1/2);
  * aligned-spin spin-orbit terms at 1.5, 2.5, 3 and 3.5PN and spin-spin terms
    at 2PN and 3PN (black-hole spin-induced quadrupole), in chi_s, chi_a;
  * tidal terms at 5PN and 6PN per body (Vines, Flanagan & Hinderer 2011),
    which sum to the -39/2 Lt v^10 and (-3115/64 Lt + 6595/364 delta dLt) v^12
    form built from the paper's Eq. (8) combinations.
Amplitude: leading order, A(f) = sqrt(5/24) pi^(-2/3) (Mc G/c^3)^(5/6)
f^(-7/6) c / (1 Mpc); no spin or tidal amplitude corrections and no
high-frequency cut-off (the ratio of the relative-binning scheme needs a
non-zero reference across the band).

Pins (tests/test_oracle_taylorf2.py): every point-particle, spin-orbit and spin-spin
coefficient is re-derived from the PN binding energy and flux (which are in turn checked
against the Kerr test-mass limit); the tidal ones against the paper's Eq. (8) form; the
amplitude against the stationary-phase amplitude of the Newtonian quadrupole chirp; the
mass conversion by the round trip from component masses.
"""
import numpy as np

from . import ad
from .constants import EULER_GAMMA, MTSUN_S, PI

V_LSO = 1.0 / np.sqrt(6.0)


def masses(mc, q):
    """Chirp mass and mass ratio q = m2/m1 -> (M_total [Msun], eta, X1, X2).

    q > 1 is allowed (labels swapped); X1 - X2 keeps its sign."""
    eta = q / (1.0 + q) ** 2
    mtot = mc * eta ** -0.6
    x1 = 1.0 / (1.0 + q)
    x2 = q / (1.0 + q)
    return mtot, eta, x1, x2


def pn_coefficients(eta, x1, x2, chi1, chi2, lam1, lam2):
    """TaylorF2 phase coefficients {k: (phi_k, phi_k^l)} in the bracket above
    (phi_k^l is None where the term has no logarithm)."""
    delta = x1 - x2
    chis = 0.5 * (chi1 + chi2)
    chia = 0.5 * (chi1 - chi2)
    eta2 = eta * eta
    eta3 = eta2 * eta
    pi2 = PI * PI

    phi2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta
    phi3 = (-16.0 * PI + 113.0 / 3.0 * delta * chia
            + (113.0 / 3.0 - 76.0 / 3.0 * eta) * chis)
    phi4 = (15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta2
            + (-405.0 / 8.0 + 200.0 * eta) * chia * chia
            - 405.0 / 4.0 * delta * chia * chis
            + (-405.0 / 8.0 + 5.0 / 2.0 * eta) * chis * chis)
    # 2.5PN: (1 + 3 ln(v/v_lso)) [pi (38645/756 - 65/9 eta) - gamma_SO]
    gamma_so = ((732985.0 / 2268.0 - 24260.0 / 81.0 * eta - 340.0 / 9.0 * eta2) * chis
                + (732985.0 / 2268.0 + 140.0 / 9.0 * eta) * delta * chia)
    c5 = PI * (38645.0 / 756.0 - 65.0 / 9.0 * eta) - gamma_so
    phi5 = c5 * (1.0 - 3.0 * np.log(V_LSO))
    phi5l = 3.0 * c5
    phi6 = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi2
            - 6848.0 / 21.0 * EULER_GAMMA - 6848.0 / 21.0 * np.log(4.0)
            + (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi2) * eta
            + 76055.0 / 1728.0 * eta2 - 127825.0 / 1296.0 * eta3
            + PI * (2270.0 / 3.0 * delta * chia + (2270.0 / 3.0 - 520.0 * eta) * chis)
            + (75515.0 / 144.0 - 8225.0 / 18.0 * eta) * delta * chia * chis
            + (75515.0 / 288.0 - 263245.0 / 252.0 * eta - 480.0 * eta2) * chia * chia
            + (75515.0 / 288.0 - 232415.0 / 504.0 * eta + 1255.0 / 9.0 * eta2) * chis * chis)
    phi6l = -6848.0 / 21.0
    phi7 = (PI * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * eta2)
            + (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta
               - 1042165.0 / 3024.0 * eta2 + 5345.0 / 36.0 * eta3) * chis
            + (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta
               - 1985.0 / 48.0 * eta2) * delta * chia)
    # Tidal, per body (A, B) = (1, 2) and (2, 1).
    phi10 = -24.0 * ((1.0 + 11.0 * x2) * x1 ** 4 * lam1 + (1.0 + 11.0 * x1) * x2 ** 4 * lam2)
    phi12 = -5.0 / 28.0 * ((3179.0 - 919.0 * x1 - 2286.0 * x1 * x1 + 260.0 * x1 ** 3) * x1 ** 4 * lam1
                           + (3179.0 - 919.0 * x2 - 2286.0 * x2 * x2 + 260.0 * x2 ** 3) * x2 ** 4 * lam2)
    return {0: (1.0, None), 2: (phi2, None), 3: (phi3, None), 4: (phi4, None),
            5: (phi5, phi5l), 6: (phi6, phi6l), 7: (phi7, None),
            10: (phi10, None), 12: (phi12, None)}


def phase(f, mc, q, chi1, chi2, lam1, lam2):
    """Psi_int(f) [rad]; parameters broadcast against f (numbers or Duals)."""
    mtot, eta, x1, x2 = masses(mc, q)
    coeffs = pn_coefficients(eta, x1, x2, chi1, chi2, lam1, lam2)
    v = ad.cbrt(PI * mtot * MTSUN_S * f)
    lnv = ad.log(v)
    bracket = 0.0
    for k, (c, cl) in coeffs.items():
        term = c if cl is None else c + cl * lnv
        bracket = bracket + (term * v ** k if k > 0 else term)
    return -PI / 4.0 + 3.0 / (128.0 * eta) * bracket / v ** 5


def amplitude(f, mc):
    """Leading-order amplitude at 1 Mpc with unit response [strain / Hz]."""
    from .constants import C_SI, MPC_M
    return (np.sqrt(5.0 / 24.0) * PI ** (-2.0 / 3.0) * (mc * MTSUN_S) ** (5.0 / 6.0)
            * f ** (-7.0 / 6.0) * (C_SI / MPC_M))
