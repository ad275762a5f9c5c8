"""Pins of the oracle's MALA step (the gradient-based local sampler of Sec. II D) against
closed forms and an exact stationarity property, and of its change of variables."""
import numpy as np
import pytest

from oracle import likelihood as L
from oracle import mala as M

from _events import near_draws, small_event


def test_linear_target_drift_is_accepted_exactly():
    """For log p = c . z and xi = 0 the proposal is z + s c / 2 and the acceptance ratio is
    exactly 1 (log alpha = s c^2/2 - (s c)^2/(2 s) = 0)."""
    c = np.array([0.7, -1.3, 2.0])
    s = np.array([0.5, 0.2, 0.1])
    z = np.array([[0.1, 0.2, 0.3], [-0.4, 0.5, -0.6]])
    lg = lambda zz: (zz @ c, np.tile(c, (len(zz), 1)))  # noqa: E731
    lp, g = lg(z)
    lo, hi = np.full(3, -10.0), np.full(3, 10.0)
    zn, lpn, gn, acc, la = M.mala_step_generic(lg, z, lp, g, s, np.zeros_like(z), np.full(2, -1e-12), lo, hi)
    np.testing.assert_allclose(zn, z + 0.5 * s * c, rtol=0, atol=1e-15)
    np.testing.assert_allclose(la, 0.0, atol=1e-14)
    assert acc.all()


def test_flat_target_proposal_is_gaussian_step():
    s = np.array([0.25, 4.0])
    z = np.zeros((3, 2))
    xi = np.array([[1.0, 0.0], [0.0, -1.0], [2.0, 0.5]])
    lg = lambda zz: (np.zeros(len(zz)), np.zeros_like(zz))  # noqa: E731
    zn, _, _, acc, la = M.mala_step_generic(lg, z, np.zeros(3), np.zeros((3, 2)), s, xi, np.full(3, -1.0), -10 * np.ones(2),
                                            10 * np.ones(2))
    np.testing.assert_allclose(zn, np.sqrt(s) * xi, rtol=1e-15)
    np.testing.assert_allclose(la, 0.0, atol=1e-15)


@pytest.mark.parametrize("step", [0.8, 1.5])
def test_gaussian_target_is_stationary(step):
    """Chains drawn from N(0, I) stay distributed as N(0, I) after one MALA step; a missing
    or reversed proposal correction moves the variance to about 0.7-0.76."""
    rng = np.random.default_rng(11)
    n, d = 400000, 2
    lg = lambda zz: (-0.5 * np.sum(zz * zz, axis=1), -zz)  # noqa: E731
    z = rng.standard_normal((n, d))
    lp, g = lg(z)
    s = np.full(d, step)
    zn, _, _, acc, _ = M.mala_step_generic(lg, z, lp, g, s, rng.standard_normal((n, d)),
                                           np.log(rng.uniform(size=n)), np.full(d, -1e9), np.full(d, 1e9))
    assert np.all(np.abs(zn.mean(axis=0)) < 0.01)
    assert np.all(np.abs(zn.var(axis=0) - 1.0) < 0.01)
    assert 0.5 < acc.mean() < 1.0


def test_box_rejects_proposals_outside_prior():
    lg = lambda zz: (np.zeros(len(zz)), np.zeros_like(zz))  # noqa: E731
    z = np.array([[0.9], [0.0]])
    zn, lpn, _, acc, _ = M.mala_step_generic(lg, z, np.zeros(2), np.zeros((2, 1)), np.array([1.0]),
                                             np.array([[0.5], [0.5]]), np.full(2, -1e300), np.array([-1.0]),
                                             np.array([1.0]))
    assert acc.tolist() == [False, True]
    assert zn[0, 0] == 0.9 and zn[1, 0] == 0.5


def test_change_of_variables_matches_differences():
    """d lnL / d cos(iota) and d lnL / d sin(dec) against central differences in z."""
    ev = small_event(duration=4.0, f_high=256.0, n_bins=30)
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 2, 31)
    z = th.copy()
    z[:, 9] = np.cos(th[:, 9])
    z[:, 12] = np.sin(th[:, 12])
    _, gz = M.loglike_grad_z(ev, z)
    for i in (9, 12, 0, 6):
        h = 1e-6 * max(1.0, abs(z[0, i]))
        zp, zm = z.copy(), z.copy()
        zp[:, i] += h
        zm[:, i] -= h
        fd = (L.loglike_rb(ev, M.z_to_theta(zp)) - L.loglike_rb(ev, M.z_to_theta(zm))) / (2 * h)
        np.testing.assert_allclose(gz[:, i], fd, rtol=2e-5, atol=1e-6 * np.abs(gz).max())


def test_mala_step_on_the_binned_likelihood_is_consistent():
    """Accepted chains carry lnL and gradient of their new position; rejected chains keep
    theirs; the decision is log u < log alpha."""
    ev = small_event(duration=4.0, f_high=256.0, n_bins=30)
    L.prepare(ev)
    th = near_draws(ev.theta_ref, 16, 32, scale=0.2)
    z = th.copy()
    z[:, 9] = np.cos(th[:, 9])
    z[:, 12] = np.sin(th[:, 12])
    lnl, gz = M.loglike_grad_z(ev, z)
    lo, hi = M.prior_box("injection")
    rng = np.random.default_rng(5)
    s = (0.1 * np.array([2e-5, 1e-2, 2e-3, 2e-3, 20.0, 20.0, 1.0, 2e-5, 0.05, 0.02, 0.02, 0.01, 0.01])) ** 2
    zn, ln, gn, acc, la = M.mala_step(ev, z, lnl, gz, s, rng.standard_normal(z.shape), np.log(rng.uniform(size=16)), lo, hi)
    l2, g2 = M.loglike_grad_z(ev, zn)
    np.testing.assert_allclose(ln, l2, rtol=1e-12)
    np.testing.assert_allclose(gn, g2, rtol=1e-10, atol=1e-10 * np.abs(g2).max())
    assert np.array_equal(zn[~acc], z[~acc])
    assert 0 < acc.sum() < 16
