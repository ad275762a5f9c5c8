"""IMRPhenomD_NRTidalv2-structured waveform (the paper's second model, Sec. II B),
as used by the oracle.

The paper names the model but prints none of it, and the calibration tables it rests
on (the IMRPhenomD phenomenological fits, the NRTidalv2 fits) are not available here.
This module therefore implements the model's *structure* with every coefficient fixed
by a stated rule (parity with the published model is unpinned):

Point-particle phase, piecewise in Mf = M f (M total mass in seconds):
  inspiral      Mf < f1 = 0.018     TaylorF2 (3.5PN point particle + aligned spins,
                                     no tidal terms), i.e. the pseudo-PN terms are zero;
  intermediate  f1 <= Mf < f2        (b0 + b1 Mf + b2 ln Mf - b3 / (3 Mf^3)) / eta,
                                     b0..b3 fixed by matching the inspiral phase and its
                                     first three derivatives at f1;
  merger-ring.  Mf >= f2 = f_RD / 2  (a0 + a1 Mf - a2 / Mf + 4/3 a3 Mf^(3/4)) / eta,
                                     a0..a3 fixed by matching the intermediate phase and
                                     its first three derivatives at f2 (the arctan term
                                     of the ringdown ansatz is left out).
Ringdown frequencies: final spin from the aligned-spin fit of Barausse & Rezzolla
(2009); radiated energy E = (1 - sqrt(8/9)) eta (test-mass binding energy at the ISCO);
quasinormal frequency and quality factor of the l = m = 2, n = 0 mode from the fits of
Berti, Cardoso & Will (2006); f_damp = f_RD / (2 Q).

Tidal phase (NRTidal Pade form): with x = (pi Mf)^(2/3) and kappa = 3/16 Lt (Lt the
paper's Eq. (8) combination),
  Psi_T = -(39/16) kappa / (X1 X2) x^(5/2) P(x),
  P = (1 + n1 x + n32 x^(3/2) + n2 x^2 + n52 x^(5/2) + n3 x^3) / (1 + d1 x + d32 x^(3/2) + d2 x^2),
whose expansion reproduces the PN tidal series 1 + c1 x + c32 x^(3/2) + c2 x^2 + c52 x^(5/2)
(c1 = 3115/1248 equals the ratio of the 6PN to 5PN TaylorF2 tidal terms).

Amplitude: A = A_0PN(f) (a_pp + a_T) w(f), with a_pp = 1 below f_peak = f_RD - f_damp
and exp(-(Mf - f_peak)/f_damp) above; tidal correction
a_T = -9 kappa x^5 (1 + 449/108 x + 22672/9 x^2.89) / (1 + 13477.8 x^4); Planck taper w
from f_merger to 1.2 f_merger (McKechan et al. 2010), with the merger frequency
M f_merger = 0.3586 / (2 pi) sqrt(X_min/X_max) (1 + 3.354e-2 kappa + 4.315e-5 kappa^2)
/ (1 + 7.542e-2 kappa + 2.236e-4 kappa^2).

Sources of the recalled constants (restated from memory of the publications; the
publications are not available here, so their equation and table numbers are not
checked, and the stand-in's parity with the published IMRPhenomD_NRTidalv2 is unpinned):
  * N52, N3, D1, D2 -- the Pade fit of the NRTidalv2 tidal phase, and the tidal amplitude
    correction (449/108, 22672/9, 2.89, 13477.8): Dietrich, Samajdar, Khan et al. 2019,
    "Improving the NRTidal model for binary neutron star systems", Phys. Rev. D 100, 044003;
  * the merger-frequency fit (0.3586, 3.354e-2, 4.315e-5, 7.542e-2, 2.236e-4): Dietrich,
    Bernuzzi & Tichy 2017 ("Closed-form tidal approximants for binary neutron star
    gravitational waveforms", Phys. Rev. D 96, 121501), as used by NRTidal;
  * S4, S5, T0, T2, T3 -- aligned-spin final-spin fit: Barausse & Rezzolla 2009, ApJ 704 L40;
  * QNM_F, QNM_Q -- l = m = 2, n = 0 fits of Berti, Cardoso & Will 2006, Phys. Rev. D 73,
    064030.
What is pinned (tests/test_oracle_nrtv2.py): the C1 region joins, the reduction to TaylorF2
below Mf = 0.018, the Pade expansion against the PN tidal series and the TaylorF2 5PN term,
zero deformability, the taper limits, the ringdown fits against Schwarzschild and the
equal-mass final spin (to the fits' accuracy), and the likelihood identities.

All functions accept numpy arrays or oracle.ad Duals for the parameters.
"""
import numpy as np

from . import ad, taylorf2
from .constants import C_SI, MPC_M, MTSUN_S, PI

F1 = 0.018
# PN tidal series and Pade fit of the NRTidal phase
C1 = 3115.0 / 1248.0
C32 = -PI
C2 = 28024205.0 / 3302208.0
C52 = -4283.0 * PI / 1092.0
N52 = 312.48173
N3 = -342.15498
D1 = -20.2372
D2 = -5.36163
# final spin (Barausse-Rezzolla 2009)
S4, S5, T0, T2, T3 = -0.1229, 0.4537, -2.8904, -3.5171, 2.5763
# l = m = 2, n = 0 quasinormal mode (Berti-Cardoso-Will 2006)
QNM_F = (1.5251, -1.1568, 0.1292)
QNM_Q = (0.7000, 1.4187, -0.4990)


def _sqrt(x):
    return ad.sqrt(x)


def kappa_tidal(x1, x2, lam1, lam2):
    """kappa = 3/16 Lt, Lt = 16/13 [(X1 + 12 X2) X1^4 L1 + (X2 + 12 X1) X2^4 L2]."""
    return (3.0 / 13.0) * ((x1 + 12.0 * x2) * x1 ** 4 * lam1 + (x2 + 12.0 * x1) * x2 ** 4 * lam2)


def pade_coefficients():
    """(n1, n32, n2, n52, n3, d1, d32, d2) of the NRTidal Pade factor."""
    d32 = (N52 - C52 - C32 * D1) / C1
    return (C1 + D1, C32 + d32, C2 + C1 * D1 + D2, N52, N3, D1, d32, D2)


def ringdown(eta, q, chi1, chi2):
    """(f_RD, f_damp) in units of 1/M (M the total mass)."""
    chit = (chi1 + q * q * chi2) / (1.0 + q * q)
    af = (chit + S4 * chit * chit * eta + S5 * chit * eta * eta + T0 * chit * eta
          + 2.0 * np.sqrt(3.0) * eta + T2 * eta * eta + T3 * eta ** 3)
    erad = (1.0 - np.sqrt(8.0 / 9.0)) * eta
    one_m = 1.0 - af
    w = QNM_F[0] + QNM_F[1] * ad.exp(QNM_F[2] * ad.log(one_m))
    qf = QNM_Q[0] + QNM_Q[1] * ad.exp(QNM_Q[2] * ad.log(one_m))
    f_rd = w / (2.0 * PI * (1.0 - erad))
    return f_rd, f_rd / (2.0 * qf)


def merger_frequency(x1, x2, kappa):
    """M f_merger of the Planck taper."""
    ratio = ad.where(ad.value(x1) >= ad.value(x2), x2 / x1, x1 / x2)
    num = 1.0 + 3.354e-2 * kappa + 4.315e-5 * kappa * kappa
    den = 1.0 + 7.542e-2 * kappa + 2.236e-4 * kappa * kappa
    return 0.3586 / (2.0 * PI) * _sqrt(ratio) * num / den


def planck_taper(f, f_start, f_end):
    """1 below f_start, 0 above f_end, 1 - 1/(exp(z) + 1) between,
    z = (f_end - f_start)/(f - f_start) + (f_end - f_start)/(f - f_end)."""
    fv = np.asarray(f, dtype=np.float64)
    fs, fe = ad.value(f_start), ad.value(f_end)
    inside = (fv > fs) & (fv < fe)
    # evaluate z only inside (placeholders elsewhere keep it finite)
    safe = np.where(inside, fv, 0.5 * (fs + fe))
    width = f_end - f_start
    z = width / (safe - f_start) + width / (safe - f_end)
    zc = np.clip(ad.value(z), -700.0, 700.0)
    wv = 1.0 - 1.0 / (np.exp(zc) + 1.0)
    # chain rule with the logistic derivative dw/dz = w (1 - w), which stays finite
    # where exp(z) and dz/dtheta are both large
    w_in = ad.Dual(wv, (wv * (1.0 - wv)) * z.d) if isinstance(z, ad.Dual) else wv
    below = fv <= fs
    return ad.where(inside, w_in, ad.where(below, np.ones_like(fv), np.zeros_like(fv)))


# --- TaylorF2 point-particle phase as a sum of powers of Mf ------------------------------

def _tf2_power_terms(eta, x1, x2, chi1, chi2):
    """Psi_TF2(Mf) = -pi/4 + sum (a x^p + b x^p ln x), x = Mf."""
    co = taylorf2.pn_coefficients(eta, x1, x2, chi1, chi2, 0.0, 0.0)
    pref = 3.0 / (128.0 * eta)
    terms = []
    for k in (0, 2, 3, 4, 5, 6, 7):
        ph, pl = co[k]
        p = (k - 5) / 3.0
        scale = PI ** p
        if pl is None:
            terms.append((pref * ph * scale, None, p))
        else:
            terms.append((pref * (ph + pl * np.log(PI) / 3.0) * scale, pref * (pl / 3.0) * scale, p))
    return terms


def _falling(p, n):
    out = 1.0
    for i in range(n):
        out *= (p - i)
    return out


def _dfalling_dp(p, n):
    # d/dp of prod_{i<n} (p - i)
    tot = 0.0
    for j in range(n):
        prod = 1.0
        for i in range(n):
            if i != j:
                prod *= (p - i)
        tot += prod
    return tot


def _tf2_derivative(terms, x, n):
    """n-th derivative with respect to Mf of Psi_TF2 at the scalar Mf = x."""
    tot = 0.0
    lx = np.log(x)
    for a, b, p in terms:
        tot = tot + a * (_falling(p, n) * x ** (p - n)) if n > 0 else tot + a * x ** p
        if b is not None:
            if n == 0:
                tot = tot + b * x ** p * lx
            else:
                s = _falling(p, n) * lx
                from math import comb, factorial
                for k in range(1, n + 1):
                    s += comb(n, k) * _falling(p, n - k) * (-1) ** (k - 1) * factorial(k - 1)
                tot = tot + b * s * x ** (p - n)
    if n == 0:
        tot = tot - PI / 4.0
    return tot


def pp_coefficients(eta, x1, x2, chi1, chi2, f2):
    """(b0..b3, a0..a3) of the intermediate and merger-ringdown phase (times eta)."""
    terms = _tf2_power_terms(eta, x1, x2, chi1, chi2)
    x = F1
    y = [eta * _tf2_derivative(terms, x, n) for n in range(4)]
    b3 = x ** 6 * (y[3] + 2.0 * y[2] / x) / 12.0
    b2 = -x * x * y[2] - 4.0 * b3 / x ** 3
    b1 = y[1] - b2 / x - b3 / x ** 4
    b0 = y[0] - b1 * x - b2 * np.log(x) + b3 / (3.0 * x ** 3)
    # intermediate form and derivatives at f2
    X = f2
    Y0 = b0 + b1 * X + b2 * ad.log(X) - b3 / (3.0 * X ** 3)
    Y1 = b1 + b2 / X + b3 / X ** 4
    Y2 = -b2 / X ** 2 - 4.0 * b3 / X ** 5
    Y3 = 2.0 * b2 / X ** 3 + 20.0 * b3 / X ** 6
    a3 = -(16.0 / 7.0) * X ** 2.25 * (Y3 + 3.0 * Y2 / X)
    a2 = -(X ** 3 / 2.0) * (Y2 + 0.25 * a3 * X ** -1.25)
    a1 = Y1 - a2 / X ** 2 - a3 * X ** -0.25
    a0 = Y0 - a1 * X + a2 / X - (4.0 / 3.0) * a3 * X ** 0.75
    return (b0, b1, b2, b3), (a0, a1, a2, a3)


def _masses(mc, q):
    mtot, eta, x1, x2 = taylorf2.masses(mc, q)
    return mtot, eta, x1, x2


def phase_pp(f, mc, q, chi1, chi2):
    """Point-particle phase [rad] (no tidal terms), piecewise in Mf."""
    mtot, eta, x1, x2 = _masses(mc, q)
    ms = mtot * MTSUN_S
    f_rd, f_damp = ringdown(eta, q, chi1, chi2)
    f2 = 0.5 * f_rd
    (b0, b1, b2, b3), (a0, a1, a2, a3) = pp_coefficients(eta, x1, x2, chi1, chi2, f2)
    mf = ms * f
    ins = taylorf2.phase(f, mc, q, chi1, chi2, 0.0, 0.0)
    inter = (b0 + b1 * mf + b2 * ad.log(mf) - b3 / (3.0 * mf ** 3)) / eta
    mr = (a0 + a1 * mf - a2 / mf + (4.0 / 3.0) * a3 * mf ** 0.75) / eta
    mfv = ad.value(mf)
    r1 = mfv < F1
    r3 = mfv >= ad.value(f2)
    return ad.where(r1, ins, ad.where(r3, mr, inter))


def phase_tidal(f, mc, q, lam1, lam2):
    """NRTidal Pade tidal phase [rad]."""
    mtot, eta, x1, x2 = _masses(mc, q)
    kap = kappa_tidal(x1, x2, lam1, lam2)
    x = (PI * mtot * MTSUN_S * f) ** (2.0 / 3.0)
    n1, n32, n2, n52, n3, d1, d32, d2 = pade_coefficients()
    sx = ad.sqrt(x)
    num = 1.0 + n1 * x + n32 * x * sx + n2 * x * x + n52 * x * x * sx + n3 * x ** 3
    den = 1.0 + d1 * x + d32 * x * sx + d2 * x * x
    return -(39.0 / 16.0) * kap / (x1 * x2) * x * x * sx * num / den


def amplitude_factor(f, mc, q, chi1, chi2, lam1, lam2, taper=True):
    """A / A_0PN = (a_pp + a_T) w."""
    mtot, eta, x1, x2 = _masses(mc, q)
    ms = mtot * MTSUN_S
    kap = kappa_tidal(x1, x2, lam1, lam2)
    f_rd, f_damp = ringdown(eta, q, chi1, chi2)
    f_peak = f_rd - f_damp
    mf = ms * f
    mfv = ad.value(mf)
    a_pp = ad.where(mfv < ad.value(f_peak), np.ones_like(mfv), ad.exp(-(mf - f_peak) / f_damp))
    x = (PI * mf) ** (2.0 / 3.0)
    a_t = -9.0 * kap * x ** 5 * (1.0 + (449.0 / 108.0) * x + (22672.0 / 9.0) * x ** 2.89) / (1.0 + 13477.8 * x ** 4)
    a = a_pp + a_t
    if taper:
        fm = merger_frequency(x1, x2, kap) / ms
        a = a * planck_taper(f, fm, 1.2 * fm)
    return a


def amplitude_phase(f, mc, q, chi1, chi2, lam1, lam2, taper=True):
    """(amplitude at 1 Mpc with unit response, Psi_int [rad])."""
    a0pn = (np.sqrt(5.0 / 24.0) * PI ** (-2.0 / 3.0) * (mc * MTSUN_S) ** (5.0 / 6.0)
            * f ** (-7.0 / 6.0) * (C_SI / MPC_M))
    amp = a0pn * amplitude_factor(f, mc, q, chi1, chi2, lam1, lam2, taper)
    psi = phase_pp(f, mc, q, chi1, chi2) + phase_tidal(f, mc, q, lam1, lam2)
    return amp, psi
