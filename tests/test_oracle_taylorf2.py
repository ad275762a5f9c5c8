"""Pins of the oracle's TaylorF2 model against physics it must reproduce.

* The point-particle and spin-orbit phase coefficients are re-derived from the
  post-Newtonian binding energy E(v) and energy flux F(v) (a separate set of
  published constants: Blanchet's review of PN theory, with the spin-orbit
  energy/flux terms of Bohe, Marsat, Faye & Blanchet 2013) through the
  stationary-phase integrals
     t(v) ~ int (5/(32 eta)) v^-9 E~(v)/F~(v) dv,
     Psi = 2 int (v^3 - v_f^3) dt/dv dv,
  so a wrong digit in either set fails.
* The 5PN/6PN tidal terms are checked against the paper's Eq. (8) combinations
  (with the second term of Lambda-tilde read as (m2 + 12 m1) m2^4 Lambda2).
* Leading-order behaviour: Psi_int(f) at v -> 0 approaches -pi/4 + 3/(128 eta v^5).
"""
import numpy as np
import pytest

from oracle import taylorf2
from oracle.constants import EULER_GAMMA

sp = pytest.importorskip("sympy")


def _derived_coefficients():
    eta, lv, d, cs, ca = sp.symbols("eta lv delta chis chia")
    pi = sp.pi
    R = sp.Rational
    S = (1 - 2 * eta) * cs + d * ca          # S_l / M^2 in chi_s, chi_a
    Sig = -d * cs - ca                       # Sigma_l / M^2
    e = {0: 1, 2: -R(3, 4) - eta / 12, 3: R(14, 3) * S + 2 * d * Sig,
         4: -R(27, 8) + R(19, 8) * eta - eta ** 2 / 24,
         5: (11 - R(61, 9) * eta) * S + d * (3 - R(10, 3) * eta) * Sig,
         6: -R(675, 64) + (R(34445, 576) - R(205, 96) * pi ** 2) * eta - R(155, 96) * eta ** 2
            - R(35, 5184) * eta ** 3,
         7: (R(135, 4) - R(367, 4) * eta + R(29, 12) * eta ** 2) * S
            + d * (R(27, 4) - 39 * eta + R(5, 4) * eta ** 2) * Sig}
    fl = {0: 1, 2: -R(1247, 336) - R(35, 12) * eta, 3: 4 * pi - 4 * S - R(5, 4) * d * Sig,
          4: -R(44711, 9072) + R(9271, 504) * eta + R(65, 18) * eta ** 2,
          5: (-R(8191, 672) - R(583, 24) * eta) * pi + (-R(9, 2) + R(272, 9) * eta) * S
             + (-R(13, 16) + R(43, 4) * eta) * d * Sig,
          6: R(6643739519, 69854400) + R(16, 3) * pi ** 2 - R(1712, 105) * sp.EulerGamma
             - R(856, 105) * (sp.log(16) + 2 * lv)
             + (-R(134543, 7776) + R(41, 48) * pi ** 2) * eta - R(94403, 3024) * eta ** 2
             - R(775, 324) * eta ** 3 - 16 * pi * S - R(31, 6) * pi * d * Sig,
          7: (-R(16285, 504) + R(214745, 1728) * eta + R(193385, 3024) * eta ** 2) * pi
             + (R(476645, 6804) + R(6172, 189) * eta - R(2810, 27) * eta ** 2) * S
             + (R(9535, 336) + R(1849, 126) * eta - R(1501, 36) * eta ** 2) * d * Sig}
    # dt/dv = 5/(32 eta) v^-9 E~/F~ with E~ = d(v^2 E)/dv / (2v).
    et = [R(k + 2, 2) * e.get(k, 0) for k in range(8)]
    ff = [fl.get(k, 0) for k in range(8)]
    inv = [sp.Integer(1)] + [0] * 7
    for k in range(1, 8):
        inv[k] = sp.expand(-sum(ff[j] * inv[k - j] for j in range(1, k + 1)))
    a = [sp.expand(sum(et[j] * inv[k - j] for j in range(k + 1))) for k in range(8)]
    # Stationary-phase integrals: v^(k-5) coefficient 40 a_k / ((k-5)(k-8));
    # ln v at k = 5 gives -40/3 a_5; at k = 6 the log term of the flux gives
    # phi_6 = -20 a_6 + 10 b_6 and phi_6^l = -20 b_6.
    b6 = a[6].coeff(lv)
    a6 = sp.expand(a[6] - b6 * lv)
    out = {k: 40 * a[k] / ((k - 5) * (k - 8)) for k in (2, 3, 4, 7)}
    out["5l"] = -R(40, 3) * a[5]
    out[6] = -20 * a6 + 10 * b6
    out["6l"] = -20 * b6
    syms = (eta, d, cs, ca)
    return {k: sp.lambdify(syms, v.subs(sp.EulerGamma, EULER_GAMMA), "math")
            for k, v in out.items()}, syms


@pytest.fixture(scope="module")
def derived():
    return _derived_coefficients()[0]


@pytest.mark.parametrize("q", [1.0, 0.8, 0.35])
@pytest.mark.parametrize("spins", [(0.04, -0.03), (-0.05, 0.02)])
def test_point_particle_and_spin_orbit_from_energy_flux(derived, q, spins):
    """Compare the spin-independent parts and the parts odd (= linear) in the
    spins; the energy/flux used carry spin-orbit terms only, and the oracle's
    coefficients are polynomials of degree <= 2 in the spins."""
    chi1, chi2 = spins
    mtot, eta, x1, x2 = taylorf2.masses(1.2, q)
    dlt = x1 - x2
    cs, ca = 0.5 * (chi1 + chi2), 0.5 * (chi1 - chi2)
    cp = taylorf2.pn_coefficients(eta, x1, x2, chi1, chi2, 0.0, 0.0)
    cm = taylorf2.pn_coefficients(eta, x1, x2, -chi1, -chi2, 0.0, 0.0)
    c0 = taylorf2.pn_coefficients(eta, x1, x2, 0.0, 0.0, 0.0, 0.0)
    for k in (2, 3, 4, 6, 7):
        want0 = derived[k](eta, dlt, 0.0, 0.0)
        assert c0[k][0] == pytest.approx(want0, rel=1e-13), k
        want_odd = 0.5 * (derived[k](eta, dlt, cs, ca) - derived[k](eta, dlt, -cs, -ca))
        got_odd = 0.5 * (cp[k][0] - cm[k][0])
        assert got_odd == pytest.approx(want_odd, rel=1e-11, abs=1e-12), k
    for k, key in ((5, "5l"), (6, "6l")):
        assert cp[k][1] == pytest.approx(derived[key](eta, dlt, cs, ca), rel=1e-12), k
    # the non-log 2.5PN part is the log part / 3 times (1 - 3 ln v_lso)
    assert cp[5][0] == pytest.approx(cp[5][1] / 3 * (1 - 3 * np.log(taylorf2.V_LSO)), rel=1e-14)


def test_tidal_terms_match_eq8_form():
    rng = np.random.default_rng(3)
    for _ in range(20):
        m1, m2 = sorted(rng.uniform(0.9, 2.6, 2))[::-1]
        l1, l2 = rng.uniform(0, 5000, 2)
        mc = (m1 * m2) ** 0.6 / (m1 + m2) ** 0.2
        mtot, eta, x1, x2 = taylorf2.masses(mc, m2 / m1)
        co = taylorf2.pn_coefficients(eta, x1, x2, 0.0, 0.0, l1, l2)
        M = m1 + m2
        lt = 16 / 13 * ((m1 + 12 * m2) * m1 ** 4 * l1 + (m2 + 12 * m1) * m2 ** 4 * l2) / M ** 5
        dlt = ((1690 / 1319 * eta - 4843 / 1319) * (m1 ** 4 * l1 - m2 ** 4 * l2) / M ** 4
               + 6162 / 1319 * np.sqrt(1 - 4 * eta) * (m1 ** 4 * l1 + m2 ** 4 * l2) / M ** 4)
        assert co[10][0] == pytest.approx(-39 / 2 * lt, rel=1e-12)
        assert co[12][0] == pytest.approx(-3115 / 64 * lt + 6595 / 364 * np.sqrt(1 - 4 * eta) * dlt,
                                          rel=1e-12)


def test_phase_leading_order_limit():
    """As f -> 0 the Newtonian term dominates: (Psi + pi/4) 128 eta v^5 / 3 -> 1."""
    mtot, eta, _, _ = taylorf2.masses(1.3, 0.7)
    from oracle.constants import MTSUN_S
    for f, tol in ((1e-3, 2e-4), (1e-5, 1e-5)):
        v = (np.pi * mtot * MTSUN_S * f) ** (1 / 3)
        psi = taylorf2.phase(np.array([f]), 1.3, 0.7, 0.01, 0.02, 100.0, 200.0)[0]
        assert (psi + np.pi / 4) * 128 * eta * v ** 5 / 3 == pytest.approx(1.0, abs=tol)


def test_tidal_phase_vanishes_without_deformability():
    f = np.linspace(20, 2048, 50)
    a = taylorf2.phase(f, 1.2, 0.9, 0.01, 0.0, 0.0, 0.0)
    b = taylorf2.phase(f, 1.2, 0.9, 0.01, 0.0, 300.0, 0.0)
    c = taylorf2.phase(f, 1.2, 0.9, 0.01, 0.0, 0.0, 0.0)
    assert np.all(a == c) and np.all(np.abs(a - b) > 0)


def test_label_swap_symmetry_of_phase():
    f = np.linspace(20, 2048, 64)
    a = taylorf2.phase(f, 1.2, 0.8, 0.03, -0.02, 300.0, 900.0)
    b = taylorf2.phase(f, 1.2, 1 / 0.8, -0.02, 0.03, 900.0, 300.0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-9)
