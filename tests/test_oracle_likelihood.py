"""Pins of the oracle's likelihood, relative binning, projection and gradient
against closed forms, invariants and brute force (no GPU)."""
import numpy as np
import pytest

import synth
from oracle import ad, binning, detector
from oracle import likelihood as L
from oracle import waveform as W
from oracle.constants import C_SI

from _events import near_draws, small_event


# ---- projection -----------------------------------------------------------------------------

def test_antenna_patterns_textbook_closed_form():
    """Arms along the Earth-frame x and y axes, gmst = 0: source polar angle
    th = pi/2 - dec and azimuth ph = ra give the textbook F+, Fx."""
    tensor = 0.5 * (np.outer([1, 0, 0], [1, 0, 0]) - np.outer([0, 1, 0], [0, 1, 0]))
    rng = np.random.default_rng(0)
    ra = rng.uniform(0, 2 * np.pi, 200)
    dec = np.arcsin(rng.uniform(-1, 1, 200))
    psi = rng.uniform(0, np.pi, 200)
    fp, fc = detector.antenna_patterns(tensor, ra, dec, psi, 0.0)
    th, ph = np.pi / 2 - dec, ra
    a = 0.5 * (1 + np.cos(th) ** 2) * np.cos(2 * ph)
    b = np.cos(th) * np.sin(2 * ph)
    np.testing.assert_allclose(fp, a * np.cos(2 * psi) - b * np.sin(2 * psi), atol=1e-14)
    np.testing.assert_allclose(fc, a * np.sin(2 * psi) + b * np.cos(2 * psi), atol=1e-14)
    # zenith: F+^2 + Fx^2 = 1 for every psi
    fp, fc = detector.antenna_patterns(tensor, 0.3, np.pi / 2, psi, 0.0)
    np.testing.assert_allclose(fp ** 2 + fc ** 2, 1.0, atol=1e-14)


def test_antenna_pattern_power_independent_of_psi():
    tensor, _ = synth.detector_geometry(0.6, -1.1, 0.7)
    psi = np.linspace(0, np.pi, 9)
    fp, fc = detector.antenna_patterns(tensor, 1.3, 0.2, psi, 0.4)
    p = fp ** 2 + fc ** 2
    np.testing.assert_allclose(p, p[0], rtol=1e-13)


def test_time_delay_closed_form():
    lat, lon = 0.4, -0.9
    _, vertex = synth.detector_geometry(lat, lon, 0.0)
    gmst = 0.25
    # source straight overhead: the wave reaches the detector R/c early
    dt = detector.time_delay(vertex, lon + gmst, lat, gmst)
    assert dt == pytest.approx(-synth.inputs.EARTH_RADIUS_M / C_SI, rel=1e-14)
    # source on the horizon (perpendicular to r): no delay
    dt = detector.time_delay(vertex, lon + gmst + np.pi / 2, 0.0, gmst)
    assert abs(dt) < 1e-20 + 1e-16 * synth.inputs.EARTH_RADIUS_M / C_SI


# ---- likelihood normalisation ---------------------------------------------------------------

def test_zero_noise_peak_is_half_hh_with_zero_gradient():
    ev = small_event(noise=False, n_bins=30)
    th0 = ev.theta_ref[None, :]
    hh = L.optimal_snr2(ev, th0)[0]
    lf, gf = L.loglike_full_grad(ev, th0)
    assert lf[0] == pytest.approx(0.5 * hh, rel=1e-12)
    lr, gr = L.loglike_rb_grad(ev, th0)
    assert lr[0] == pytest.approx(0.5 * hh, rel=1e-12)
    scale = np.abs(L.loglike_full_grad(ev, near_draws(ev.theta_ref, 1, 1))[1]).max()
    assert np.abs(gf).max() <= 1e-9 * scale
    assert np.abs(gr).max() <= 1e-9 * scale


def test_rb_equals_full_at_reference():
    """r == 1 at theta0: r0 = 1, r1 = 0, sum A0 = <d, h0>_c, sum B0 = <h0, h0>."""
    ev = small_event(n_bins=25)
    th0 = ev.theta_ref[None, :]
    L.prepare(ev)
    full = L.loglike_full(ev, th0)[0]
    rb = L.loglike_rb(ev, th0)[0]
    assert rb == pytest.approx(full, rel=1e-12)
    h0 = W.strain(ev.f, th0, ev.tensors, ev.vertices, ev.gmst, ev.approximant, False)
    for d in range(len(h0)):
        assert ev.summary["A0"][d].sum() == pytest.approx(
            L.inner_c(ev.data[d], h0[d][0], ev.psd[d], ev.delta_f), rel=1e-12)
        assert ev.summary["B0"][d].sum() == pytest.approx(
            L.inner_c(h0[d][0], h0[d][0], ev.psd[d], ev.delta_f).real, rel=1e-12)


def test_rb_one_bin_per_grid_point_is_exact_with_b2():
    """Edges at every grid point: the piecewise-linear model is exact at the
    grid points, so with B2 kept the binned lnL equals the full one anywhere."""
    ev = small_event(duration=1.0, f_high=300.0, keep_b2=True)
    ev.edges = np.arange(len(ev.f))
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 6, 3, scale=20.0)
    np.testing.assert_allclose(L.loglike_rb(ev, th), L.loglike_full(ev, th), rtol=1e-11)


def test_rb_converges_to_full_under_refinement():
    ev = small_event(duration=8.0, f_high=1024.0)
    th = near_draws(ev.theta_ref, 8, 5)
    full = L.loglike_full(ev, th)
    errs = []
    for nb in (25, 50, 100, 200, 400):
        ev.edges = binning.pn_bin_edges(ev.f[0], ev.delta_f, len(ev.f), nb)
        L.prepare(ev)
        errs.append(np.abs(L.loglike_rb(ev, th) - full).max())
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0), errs
    slope = np.polyfit(np.log([25, 50, 100, 200, 400]), np.log(errs), 1)[0]
    assert slope < -1.5, slope


def test_label_swap_invariance():
    ev = small_event()
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 5, 9)
    sw = th.copy()
    sw[:, 1] = 1.0 / th[:, 1]
    sw[:, [2, 3]] = th[:, [3, 2]]
    sw[:, [4, 5]] = th[:, [5, 4]]
    np.testing.assert_allclose(L.loglike_rb(ev, sw), L.loglike_rb(ev, th), rtol=1e-10)
    np.testing.assert_allclose(L.loglike_full(ev, sw), L.loglike_full(ev, th), rtol=1e-10)


def test_phase_and_polarisation_degeneracy():
    ev = small_event()
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 5, 11)
    a = L.loglike_rb(ev, th)
    t2 = th.copy()
    t2[:, 8] += np.pi
    np.testing.assert_allclose(L.loglike_rb(ev, t2), a, rtol=1e-10)
    t3 = th.copy()
    t3[:, 8] += np.pi / 2
    t3[:, 10] += np.pi / 2
    np.testing.assert_allclose(L.loglike_rb(ev, t3), a, rtol=1e-10)


def test_distance_closed_form():
    """lnL(dL) = a/dL - b/(2 dL^2): two distances fix a, b; two more are predicted."""
    ev = small_event()
    L.prepare(ev)
    base = near_draws(ev.theta_ref, 1, 13)[0]
    ds = np.array([20.0, 45.0, 80.0, 150.0])
    th = np.tile(base, (4, 1))
    th[:, 6] = ds
    for fn in (L.loglike_rb, L.loglike_full):
        v = fn(ev, th)
        m = np.stack([1 / ds[:2], -0.5 / ds[:2] ** 2], 1)
        a, b = np.linalg.solve(m, v[:2])
        np.testing.assert_allclose(v[2:], a / ds[2:] - b / (2 * ds[2:] ** 2), rtol=1e-10)


def test_phase_and_distance_gradient_closed_forms():
    """d lnL/d phic = 2 Im z, d lnL/d dL = (-Re z + <h, h>)/dL with
    z = sum_d <d, h>_c (binned: the same with the binned sums)."""
    ev = small_event()
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 3, 17)
    _, g = L.loglike_full_grad(ev, th)
    hs = W.strain(ev.f, th, ev.tensors, ev.vertices, ev.gmst, ev.approximant)
    z = sum(L.inner_c(ev.data[d], hs[d], ev.psd[d], ev.delta_f) for d in range(len(hs)))
    hh = L.optimal_snr2(ev, th)
    np.testing.assert_allclose(g[:, 8], 2 * z.imag, rtol=1e-10)
    np.testing.assert_allclose(g[:, 6], (-z.real + hh) / th[:, 6], rtol=1e-10)
    # binned: z_RB = sum A0 r0* + A1 r1*, hh_RB = sum B0|r0|^2 + 2 B1 Re(r0 r1*)
    _, gr = L.loglike_rb_grad(ev, th)
    s = ev.summary
    fn = ev.f[ev.edges]
    zr, hr = 0.0, 0.0
    for d, r in enumerate(L.node_ratios(ev, th)):
        r0 = 0.5 * (r[:, 1:] + r[:, :-1])
        r1 = (r[:, 1:] - r[:, :-1]) / (fn[1:] - fn[:-1])
        zr = zr + (s["A0"][d] * np.conj(r0) + s["A1"][d] * np.conj(r1)).sum(-1)
        hr = hr + (s["B0"][d] * np.abs(r0) ** 2 + 2 * s["B1"][d] * (r0 * np.conj(r1)).real).sum(-1)
    np.testing.assert_allclose(gr[:, 8], 2 * zr.imag, rtol=1e-10)
    np.testing.assert_allclose(gr[:, 6], (-zr.real + hr) / th[:, 6], rtol=1e-10)


def test_dual_gradient_matches_central_differences():
    ev = small_event()
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 2, 19)
    _, g = L.loglike_rb_grad(ev, th)
    width = np.array([0.03, 0.875, 0.1, 0.1, 5000, 5000, 74, 0.2, 2 * np.pi, np.pi, np.pi,
                      2 * np.pi, np.pi])
    for i in range(13):
        h = 1e-6 * np.maximum(np.abs(th[:, i]), width[i])
        tp, tm = th.copy(), th.copy()
        tp[:, i] += h
        tm[:, i] -= h
        fd = (L.loglike_rb(ev, tp) - L.loglike_rb(ev, tm)) / (2 * h)
        # Richardson with h/2 removes the O(h^2) term
        tp2, tm2 = th.copy(), th.copy()
        tp2[:, i] += h / 2
        tm2[:, i] -= h / 2
        fd2 = (L.loglike_rb(ev, tp2) - L.loglike_rb(ev, tm2)) / h
        rich = (4 * fd2 - fd) / 3
        scale = np.abs(g * width).max(axis=1)
        err = np.abs((rich - g[:, i]) * width[i])
        assert np.all(err <= 1e-5 * scale), (i, err / scale)


# ---- noise ---------------------------------------------------------------------------------

def test_noise_statistics():
    """Over many seeds: E<n, n> = 2 N per detector and Var Re<n, h>_c = <h, h>."""
    f_low, delta_f, n, f = synth.frequency_grid(20.0, 100.0, 4.0)
    psd = synth.analytic_psd(f)[None, :]
    h = (1e-23 * np.exp(1j * f / 10.0))[None, :]
    hh = L.inner_c(h[0], h[0], psd[0], delta_f).real
    nn, nh = [], []
    for s in range(1000):
        nz = synth.gaussian_noise(s, psd, 4.0)[0]
        nn.append(L.inner_c(nz, nz, psd[0], delta_f).real)
        nh.append(L.inner_c(nz, h[0], psd[0], delta_f).real)
    nn, nh = np.array(nn), np.array(nh)
    assert abs(nn.mean() - 2 * n) < 3 * nn.std() / np.sqrt(len(nn))
    # variance estimate: relative standard error sqrt(2/(k-1))
    assert abs(nh.var() / hh - 1) < 3 * np.sqrt(2 / 999)


def test_dual_numbers_against_closed_forms():
    x, y = ad.seed([0.7, 1.9])
    z = ad.exp(1j * x) * y ** 2.5 / ad.cbrt(x) + ad.arctan(x * y) - ad.sqrt(y) * ad.log(x)
    dzdx = (1j * np.exp(0.7j) * 1.9 ** 2.5 / 0.7 ** (1 / 3)
            - np.exp(0.7j) * 1.9 ** 2.5 / (3 * 0.7 ** (4 / 3))
            + 1.9 / (1 + (0.7 * 1.9) ** 2) - np.sqrt(1.9) / 0.7)
    dzdy = (2.5 * np.exp(0.7j) * 1.9 ** 1.5 / 0.7 ** (1 / 3) + 0.7 / (1 + (0.7 * 1.9) ** 2)
            - 0.5 / np.sqrt(1.9) * np.log(0.7))
    assert z.d[0] == pytest.approx(dzdx, rel=1e-14)
    assert z.d[1] == pytest.approx(dzdy, rel=1e-14)


# ---- centre-node variant of Eq. (5) -----------------------------------------------------------

def _brute_piecewise_linear(ev, th, centre):
    """Full-grid likelihood of the piecewise-linear model h = h0 (r0 + r1 (f - f_m)) per bin,
    written directly on the grid (no summary data), minus nothing: returns (lnL_model, S2)
    with S2 = sum_b B2 |r1|^2 / 2 computed on the grid, so that the binned formula without
    the B2 term equals lnL_model + S2."""
    edges = np.asarray(ev.edges)
    f = ev.f
    fe = f[edges]
    fm = 0.5 * (fe[:-1] + fe[1:])
    b_of_k = L.bin_index(len(f), edges)
    h0 = W.strain(f, ev.theta_ref, ev.tensors, ev.vertices, ev.gmst, ev.approximant, ev.ref_taper)
    r_e = L.node_ratios(ev, th)
    r_c = L.node_ratios(ev, th, fm) if centre else None
    out, s2 = 0.0, 0.0
    for d in range(len(h0)):
        rl, rr = r_e[d][:, :-1], r_e[d][:, 1:]
        r0 = r_c[d] if centre else 0.5 * (rl + rr)
        r1 = (rr - rl) / (fe[1:] - fe[:-1])
        model = h0[d][0] * (r0[:, b_of_k] + r1[:, b_of_k] * (f - fm[b_of_k]))
        w = 4.0 * ev.delta_f / ev.psd[d]
        out = out + (np.conj(model) * ev.data[d] * w).sum(-1).real - 0.5 * (np.abs(model) ** 2 * w).sum(-1)
        q = np.abs(h0[d][0]) ** 2 * w * (f - fm[b_of_k]) ** 2
        b2 = np.array([q[b_of_k == b].sum() for b in range(len(fm))])
        s2 = s2 + 0.5 * (b2 * np.abs(r1) ** 2).sum(-1)
    return out, s2


@pytest.mark.parametrize("approximant", ["taylorf2", "phenomd_nrtv2"])
def test_centre_variant_equals_its_piecewise_linear_model(approximant):
    """The binned sum with r0 = r(f_m) is the full-grid likelihood of the piecewise-linear
    ratio through r(f_m) with the edge slope, up to its dropped B2 term (brute force)."""
    ev = small_event(approximant=approximant, duration=2.0, f_high=400.0, n_bins=30)
    ev.centre = True
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 4, 31, scale=5.0)
    model, s2 = _brute_piecewise_linear(ev, th, centre=True)
    np.testing.assert_allclose(L.loglike_rb(ev, th), model + s2, rtol=1e-11)
    # and the edge variant matches its own model the same way (the two differ)
    ev.centre = False
    model_e, s2_e = _brute_piecewise_linear(ev, th, centre=False)
    np.testing.assert_allclose(L.loglike_rb(ev, th), model_e + s2_e, rtol=1e-11)
    assert np.abs(model - model_e).max() > 1e-6 * np.abs(model).max()


def test_centre_variant_exact_at_reference_and_converges():
    ev = small_event(duration=8.0, f_high=1024.0)
    ev.centre = True
    th0 = ev.theta_ref[None, :]
    th = near_draws(ev.theta_ref, 8, 5)
    full, full0 = L.loglike_full(ev, th), L.loglike_full(ev, th0)[0]
    errs = []
    for nb in (25, 50, 100, 200, 400):
        ev.edges = binning.pn_bin_edges(ev.f[0], ev.delta_f, len(ev.f), nb)
        L.prepare(ev)
        assert L.loglike_rb(ev, th0)[0] == pytest.approx(full0, rel=1e-12)
        errs.append(np.abs(L.loglike_rb(ev, th) - full).max())
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0), errs
    slope = np.polyfit(np.log([25, 50, 100, 200, 400]), np.log(errs), 1)[0]
    assert slope < -1.5, slope


def test_centre_variant_refuses_b2():
    ev = small_event(keep_b2=True)
    ev.centre = True
    with pytest.raises(ValueError):
        L.loglike_rb(ev, ev.theta_ref[None, :])
