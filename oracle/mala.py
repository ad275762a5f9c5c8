"""One Metropolis-adjusted Langevin (MALA) step for a batch of chains: the local sampler
the paper's pipeline drives with the likelihood gradient (Sec. II D), over the uniform
priors of Tab. II.  Test infrastructure, like the rest of the oracle.

Sampled coordinates z (13): (Mc, q, chi1, chi2, Lambda1, Lambda2, dL, tc, phic, cos iota,
psi, ra, sin delta) -- the variables in which Tab. II's priors are uniform.  The target is
log p(z) = lnL(theta(z)) inside the prior box and -inf outside (a uniform prior adds only a
constant).  With a diagonal step s (s_i = eps^2 M_ii):

  proposal   z' = z + (s / 2) g(z) + sqrt(s) xi,          xi ~ N(0, 1)
  log q(b|a) = -sum_i (b_i - a_i - s_i g_i(a) / 2)^2 / (2 s_i)   (+ const)
  accept     if log u < log p(z') - log p(z) + log q(z|z') - log q(z'|z)

where g = d log p / dz.  The random numbers xi [B, 13] and log u [B] are inputs.
"""
import numpy as np

from . import likelihood as L

IOTA, DEC = 9, 12


def z_to_theta(z):
    """Sampled coordinates -> the 13 likelihood parameters (iota, dec as angles)."""
    z = np.atleast_2d(np.asarray(z, dtype=np.float64))
    th = z.copy()
    th[:, IOTA] = np.arccos(np.clip(z[:, IOTA], -1.0, 1.0))
    th[:, DEC] = np.arcsin(np.clip(z[:, DEC], -1.0, 1.0))
    return th


def grad_theta_to_z(theta, g):
    """Chain rule d lnL/dz from d lnL/dtheta: d/dcos(iota) = -(d/diota) / sin(iota),
    d/dsin(dec) = (d/ddec) / cos(dec)."""
    gz = np.array(g, dtype=np.float64, copy=True)
    gz[:, IOTA] = -g[:, IOTA] / np.sin(theta[:, IOTA])
    gz[:, DEC] = g[:, DEC] / np.cos(theta[:, DEC])
    return gz


def in_box(z, lo, hi):
    return np.all((z >= lo) & (z <= hi), axis=1)


def log_q(b, a, ga, s):
    """log q(b | a) of the Langevin proposal (without its constant)."""
    r = b - a - 0.5 * s * ga
    return -np.sum(r * r / (2.0 * s), axis=1)


def mala_step_generic(logp_grad, z, logp, g, s, xi, logu, lo, hi):
    """One MALA step for any target.  logp_grad(z') -> (log p, gradient) for proposals
    inside the box.  Returns (z_new, logp_new, g_new, accepted)."""
    z = np.atleast_2d(z)
    zp = z + 0.5 * s * g + np.sqrt(s) * xi
    inside = in_box(zp, lo, hi)
    lp = np.full(len(z), -np.inf)
    gp = np.zeros_like(z)
    if inside.any():
        lpi, gpi = logp_grad(zp[inside])
        lp[inside] = lpi
        gp[inside] = gpi
    with np.errstate(invalid="ignore"):
        log_alpha = lp - logp + log_q(z, zp, gp, s) - log_q(zp, z, g, s)
    acc = inside & np.isfinite(lp) & (logu < log_alpha)
    z_new = np.where(acc[:, None], zp, z)
    logp_new = np.where(acc, lp, logp)
    g_new = np.where(acc[:, None], gp, g)
    return z_new, logp_new, g_new, acc, log_alpha


def loglike_grad_z(ev, z):
    """lnL and d lnL / dz of the relative-binned likelihood at sampled coordinates z."""
    th = z_to_theta(z)
    lnl, g = L.loglike_rb_grad(ev, th)
    return lnl, grad_theta_to_z(th, g)


def mala_step(ev, z, lnl, gz, s, xi, logu, lo, hi):
    """One MALA step of B chains on the binned likelihood of event ev (Sec. II D)."""
    return mala_step_generic(lambda zz: loglike_grad_z(ev, zz), z, lnl, gz, s, xi, logu, lo, hi)


def prior_box(column):
    """Tab. II bounds in the sampled coordinates for a prior column of synth.PRIORS."""
    import synth
    b = synth.PRIORS[column]
    lo = np.array([b["Mc"][0], b["q"][0], b["chi"][0], b["chi"][0], b["L"][0], b["L"][0], b["dL"][0], b["tc"][0],
                   0.0, -1.0, 0.0, 0.0, -1.0])
    hi = np.array([b["Mc"][1], b["q"][1], b["chi"][1], b["chi"][1], b["L"][1], b["L"][1], b["dL"][1], b["tc"][1],
                   2 * np.pi, 1.0, np.pi, 2 * np.pi, 1.0])
    return lo, hi
