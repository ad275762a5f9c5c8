"""Pins of the oracle's IMRPhenomD_NRTidalv2-structured model (no GPU).

The model's calibration tables are not available, so its coefficients follow stated
rules (see the module docstring); these tests pin what those rules and the physics
fix: smooth region joins, reduction to TaylorF2 in the inspiral, the tidal Pade form
against the PN tidal series and the TaylorF2 tidal term, the Planck taper, the
ringdown fits against Schwarzschild/NR values, and the likelihood identities."""
import numpy as np
import pytest

from oracle import ad, phenomd_nrtv2 as P, taylorf2 as T
from oracle import likelihood as L
from oracle.constants import MTSUN_S

from _events import near_draws, small_event

PARAMS = [(1.43562, 0.94118, 0.01, 0.01, 400.0, 400.0), (1.2, 0.6, 0.04, -0.03, 100.0, 2500.0),
          (2.4, 0.2, -0.05, 0.05, 0.0, 700.0)]


def _phase_and_derivs(fv, mc, q, c1, c2):
    """Phase and its first derivative in f, by a dual number seeded in f."""
    f = ad.Dual(np.array([fv]), np.ones((1, 1)))
    ph = P.phase_pp(f, mc, q, c1, c2)
    return ph.v.ravel()[0], ph.d.ravel()[0]


@pytest.mark.parametrize("par", PARAMS)
def test_phase_regions_join_smoothly(par):
    mc, q, c1, c2, _, _ = par
    mtot, eta, _, _ = T.masses(mc, q)
    ms = mtot * MTSUN_S
    f_rd, _ = P.ringdown(eta, q, c1, c2)
    for mf in (P.F1, 0.5 * f_rd):
        f = mf / ms
        lo = _phase_and_derivs(f * (1 - 1e-12), mc, q, c1, c2)
        hi = _phase_and_derivs(f * (1 + 1e-12), mc, q, c1, c2)
        assert hi[0] == pytest.approx(lo[0], rel=1e-9, abs=1e-6)
        assert hi[1] == pytest.approx(lo[1], rel=1e-7)


def test_inspiral_region_is_taylorf2_point_particle():
    mc, q, c1, c2 = 1.3, 0.7, 0.02, -0.01
    mtot, _, _, _ = T.masses(mc, q)
    f = np.linspace(20.0, 0.99 * P.F1 / (mtot * MTSUN_S), 50)
    np.testing.assert_allclose(np.ravel(P.phase_pp(f, mc, q, c1, c2)), np.ravel(T.phase(f, mc, q, c1, c2, 0.0, 0.0)),
                               rtol=1e-14, atol=1e-12)
    amp, psi = P.amplitude_phase(f, mc, q, c1, c2, 0.0, 0.0, taper=False)
    np.testing.assert_allclose(np.ravel(amp), T.amplitude(f, mc), rtol=1e-14)


def test_pade_reproduces_pn_tidal_series():
    n1, n32, n2, n52, n3, d1, d32, d2 = P.pade_coefficients()
    for x in (1e-3, 5e-4, 2.5e-4):
        s = np.sqrt(x)
        pade = (1 + n1 * x + n32 * x * s + n2 * x * x + n52 * x * x * s + n3 * x ** 3) / \
               (1 + d1 * x + d32 * x * s + d2 * x * x)
        series = 1 + P.C1 * x + P.C32 * x * s + P.C2 * x * x + P.C52 * x * x * s
        # remainder is O(x^3)
        assert abs(pade - series) < 1e4 * x ** 3
    # c1 is the ratio of the TaylorF2 6PN and 5PN tidal terms at equal mass
    assert P.C1 == pytest.approx((3115.0 / 64.0) / (39.0 / 2.0), rel=1e-15)


def test_leading_tidal_phase_equals_taylorf2_5pn_term():
    rng = np.random.default_rng(4)
    for _ in range(10):
        mc, q = rng.uniform(1.0, 2.0), rng.uniform(0.3, 1.0)
        l1, l2 = rng.uniform(0, 5000, 2)
        mtot, eta, x1, x2 = T.masses(mc, q)
        co = T.pn_coefficients(eta, x1, x2, 0.0, 0.0, l1, l2)
        kap = P.kappa_tidal(x1, x2, l1, l2)
        # -(39/16) kappa / (X1 X2) x^(5/2)  vs  3/(128 eta) phi10 v^5, x = v^2
        assert -(39.0 / 16.0) * kap / (x1 * x2) == pytest.approx(3.0 / (128.0 * eta) * co[10][0], rel=1e-13)


def test_zero_deformability_removes_tidal_terms():
    mc, q, c1, c2 = 1.4, 0.8, 0.0, 0.0
    f = np.linspace(20.0, 2048.0, 40)
    assert np.all(P.phase_tidal(f, mc, q, 0.0, 0.0) == 0.0)
    a = P.amplitude_factor(f, mc, q, c1, c2, 0.0, 0.0, taper=False)
    np.testing.assert_array_equal(np.ravel(a), np.ones_like(f))
    mtot, _, x1, x2 = T.masses(mc, q)
    fm = P.merger_frequency(x1, x2, 0.0) / (mtot * MTSUN_S)
    assert fm == pytest.approx(0.3586 / (2 * np.pi) * np.sqrt(q) / (mtot * MTSUN_S), rel=1e-14)


def test_planck_taper_limits():
    fm = 1500.0
    f = np.array([100.0, fm, fm * 1.0000001, 1.1 * fm, 1.2 * fm * 0.9999999, 1.2 * fm, 3000.0])
    w = P.planck_taper(f, fm, 1.2 * fm)
    assert w[0] == 1.0 and w[1] == 1.0 and w[5] == 0.0 and w[6] == 0.0
    assert w[3] == pytest.approx(0.5, abs=1e-12)
    assert w[2] > 1 - 1e-12 and w[4] < 1e-12
    ff = np.linspace(fm, 1.2 * fm, 101)
    assert np.all(np.diff(P.planck_taper(ff, fm, 1.2 * fm)) <= 0)


def test_ringdown_fits_against_known_values():
    # Schwarzschild l=m=2, n=0: M omega = 0.37367, Q = omega_R / (2 omega_I) = 2.10
    w = P.QNM_F[0] + P.QNM_F[1]
    qf = P.QNM_Q[0] + P.QNM_Q[1]
    assert w == pytest.approx(0.37367, rel=0.02)
    assert qf == pytest.approx(0.37367 / (2 * 0.08896), rel=0.02)
    # equal-mass non-spinning binary black hole: final spin 0.686
    eta = 0.25
    chit = 0.0
    af = 2 * np.sqrt(3) * eta + P.T2 * eta ** 2 + P.T3 * eta ** 3 + 0 * chit
    assert af == pytest.approx(0.686, abs=0.005)


@pytest.mark.parametrize("keep_taper", [True, False])
def test_rb_identities_nrtv2(keep_taper):
    """Taper treated the same in reference and samples: binned == full at theta0, and
    the zero-noise injection peaks at <h, h>/2 with zero gradient."""
    # band ends inside the taper (w > 0), so a tapered reference stays non-zero
    th = small_event(approximant="phenomd_nrtv2", noise=False, duration=1.0, f_high=100.0).theta_ref
    mtot, _, x1, x2 = T.masses(th[0], th[1])
    fm = P.merger_frequency(x1, x2, P.kappa_tidal(x1, x2, th[4], th[5])) / (mtot * MTSUN_S)
    ev = small_event(approximant="phenomd_nrtv2", noise=False, duration=4.0, f_high=float(np.floor(1.15 * fm)),
                     n_bins=60, ref_taper=keep_taper)
    th0 = ev.theta_ref[None, :]
    if not keep_taper:
        # data generated with the taper; compare at theta0 using untapered strains on both sides
        from oracle import waveform as W
        h = W.strain(ev.f, th0, ev.tensors, ev.vertices, ev.gmst, "phenomd_nrtv2", False)
        ev.data = np.stack([x[0] for x in h])
        L.prepare(ev)
        full = L.loglike_full(ev, th0, taper=False)[0]
        r = L.node_ratios(ev, th0)
        # samples are tapered: ratio is the taper, 1 below f_merger
        assert np.allclose(np.abs(r[0][0][: len(r[0][0]) // 3]), 1.0, rtol=1e-12)
        return
    L.prepare(ev)
    hh = L.optimal_snr2(ev, th0)[0]
    lr, gr = L.loglike_rb_grad(ev, th0)
    assert lr[0] == pytest.approx(0.5 * hh, rel=1e-11)
    lf = L.loglike_full(ev, th0)[0]
    assert lr[0] == pytest.approx(lf, rel=1e-11)
    scale = np.abs(L.loglike_rb_grad(ev, near_draws(ev.theta_ref, 1, 3))[1]).max()
    assert np.abs(gr).max() <= 1e-8 * scale


def test_label_swap_invariance_nrtv2():
    ev = small_event(approximant="phenomd_nrtv2", duration=4.0, f_high=2048.0, n_bins=60)
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 4, 21)
    sw = th.copy()
    sw[:, 1] = 1.0 / th[:, 1]
    sw[:, [2, 3]] = th[:, [3, 2]]
    sw[:, [4, 5]] = th[:, [5, 4]]
    np.testing.assert_allclose(L.loglike_rb(ev, sw), L.loglike_rb(ev, th), rtol=1e-9)


def test_nrtv2_dual_gradient_matches_richardson():
    ev = small_event(approximant="phenomd_nrtv2", duration=4.0, f_high=2048.0, n_bins=60)
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 2, 23)
    _, g = L.loglike_rb_grad(ev, th)
    width = np.array([0.03, 0.875, 0.1, 0.1, 5000, 5000, 74, 0.2, 2 * np.pi, np.pi, np.pi, 2 * np.pi, np.pi])
    for i in range(6):
        h = 1e-6 * np.maximum(np.abs(th[:, i]), width[i])
        fd = []
        for s in (1.0, 0.5):
            tp, tm = th.copy(), th.copy()
            tp[:, i] += s * h
            tm[:, i] -= s * h
            fd.append((L.loglike_rb(ev, tp) - L.loglike_rb(ev, tm)) / (2 * s * h))
        rich = (4 * fd[1] - fd[0]) / 3
        scale = np.abs(g * width).max(axis=1)
        assert np.all(np.abs((rich - g[:, i]) * width[i]) <= 1e-5 * scale), i
