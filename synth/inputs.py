"""Seeded generators of the likelihood's inputs (no method arithmetic).

Parameter order (Tab. II of the paper, with the inclination and declination
carried as angles rather than their cosine / sine):
    0 Mc   detector-frame chirp mass [Msun]
    1 q    mass ratio m2/m1 (<= 1 for the prior, > 1 allowed for label swaps)
    2 chi1 aligned spin of body 1
    3 chi2 aligned spin of body 2
    4 L1   dimensionless tidal deformability of body 1
    5 L2   dimensionless tidal deformability of body 2
    6 dL   luminosity distance [Mpc]
    7 tc   coalescence time [s]
    8 phic coalescence (orbital) phase [rad]
    9 iota inclination [rad]
   10 psi  polarisation angle [rad]
   11 ra   right ascension [rad]
   12 dec  declination [rad]
"""
import numpy as np

PARAM_NAMES = ("Mc", "q", "chi1", "chi2", "L1", "L2", "dL", "tc", "phic",
               "iota", "psi", "ra", "dec")
N_PARAMS = len(PARAM_NAMES)

# Uniform prior boxes of Tab. II.  cos(iota) and sin(dec) are uniform in
# [-1, 1]; the draws below convert them to angles.
PRIORS = {
    "injection": {"Mc": (0.88, 2.61), "q": (0.5, 1.0), "chi": (-0.05, 0.05),
                  "L": (0.0, 5000.0), "dL": (30.0, 300.0), "tc": (-0.1, 0.1)},
    "gw170817": {"Mc": (1.18, 1.21), "q": (0.125, 1.0), "chi": (-0.05, 0.05),
                 "L": (0.0, 5000.0), "dL": (1.0, 75.0), "tc": (-0.1, 0.1)},
    "gw190425": {"Mc": (1.485, 1.490), "q": (0.125, 1.0), "chi": (-0.05, 0.05),
                 "L": (0.0, 5000.0), "dL": (1.0, 500.0), "tc": (-0.1, 0.1)},
}


def frequency_grid(f_low, f_high, duration):
    """Uniform grid f_k = f_low + k/T, both band ends included.

    Returns (f_low, delta_f, n_freq, f) with f the float64 grid.
    """
    delta_f = 1.0 / duration
    n_freq = int(round((f_high - f_low) * duration)) + 1
    f = f_low + delta_f * np.arange(n_freq, dtype=np.float64)
    return f_low, delta_f, n_freq, f


def analytic_psd(f):
    """One-sided analytic PSD used by every workload (a design-sensitivity
    stand-in): S(f) = 1e-49 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2)/(1 + x^2/2)],
    x = f / 215 Hz."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    return 1e-49 * (x ** -4.14 - 5.0 * x ** -2
                    + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


EARTH_RADIUS_M = 6378137.0


def detector_geometry(lat, lon, azimuth):
    """Long-wavelength L-shaped interferometer on a spherical Earth.

    The x arm points at `azimuth` (radians east of local north), the y arm 90
    degrees further (x = cos(b) N + sin(b) E, y = -sin(b) N + cos(b) E).
    Returns the Earth-fixed detector tensor D = (xx^T - yy^T)/2 (3x3) and the
    vertex position [m].
    """
    e_north = np.array([-np.sin(lat) * np.cos(lon), -np.sin(lat) * np.sin(lon), np.cos(lat)])
    e_east = np.array([-np.sin(lon), np.cos(lon), 0.0])
    x = np.cos(azimuth) * e_north + np.sin(azimuth) * e_east
    y = -np.sin(azimuth) * e_north + np.cos(azimuth) * e_east
    tensor = 0.5 * (np.outer(x, x) - np.outer(y, y))
    vertex = EARTH_RADIUS_M * np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
    return tensor, vertex


def gaussian_noise(seed, psd, duration):
    """Stationary Gaussian noise in the frequency domain.

    Re and Im of each sample are independent N(0, T S / 4), so that the noise
    inner product has expectation 2 per frequency sample.  psd has shape
    [n_det, n_freq]; detectors are drawn in order, real block then imaginary
    block, from one PCG64 stream.
    """
    psd = np.atleast_2d(np.asarray(psd, dtype=np.float64))
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(psd.shape, dtype=np.complex128)
    for d in range(psd.shape[0]):
        sigma = np.sqrt(duration * psd[d] / 4.0)
        re = rng.standard_normal(psd.shape[1]) * sigma
        im = rng.standard_normal(psd.shape[1]) * sigma
        out[d] = re + 1j * im
    return out


def draw_theta(seed, n, prior, mc_window=None):
    """n parameter vectors drawn from a Tab. II uniform prior (float64 [n, 13]).

    `mc_window` = (lo, hi) overrides the chirp-mass range (used to recentre a
    narrow window on an injection).
    """
    box = PRIORS[prior]
    mc = mc_window if mc_window is not None else box["Mc"]
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.empty((n, N_PARAMS), dtype=np.float64)
    th[:, 0] = rng.uniform(*mc, n)
    th[:, 1] = rng.uniform(*box["q"], n)
    th[:, 2] = rng.uniform(*box["chi"], n)
    th[:, 3] = rng.uniform(*box["chi"], n)
    th[:, 4] = rng.uniform(*box["L"], n)
    th[:, 5] = rng.uniform(*box["L"], n)
    th[:, 6] = rng.uniform(*box["dL"], n)
    th[:, 7] = rng.uniform(*box["tc"], n)
    th[:, 8] = rng.uniform(0.0, 2 * np.pi, n)
    th[:, 9] = np.arccos(rng.uniform(-1.0, 1.0, n))
    th[:, 10] = rng.uniform(0.0, np.pi, n)
    th[:, 11] = rng.uniform(0.0, 2 * np.pi, n)
    th[:, 12] = np.arcsin(rng.uniform(-1.0, 1.0, n))
    return th


def mismatch_draws(seed, n):
    """n parameter vectors of the waveform-accuracy study (the paper's Tab. I): component
    masses uniform in [0.5, 3] Msun (either may be the heavier: q = m2/m1 may exceed 1),
    aligned spins uniform in [-0.05, 0.05], tidal deformabilities uniform in [0, 5000],
    inclination uniform in [0, pi]; distance 100 Mpc and the remaining angles fixed
    (the mismatch does not depend on them)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m1 = rng.uniform(0.5, 3.0, n)
    m2 = rng.uniform(0.5, 3.0, n)
    mc, q = component_to_chirp(m1, m2)
    th = np.empty((n, N_PARAMS), dtype=np.float64)
    th[:, 0], th[:, 1] = mc, q
    th[:, 2] = rng.uniform(-0.05, 0.05, n)
    th[:, 3] = rng.uniform(-0.05, 0.05, n)
    th[:, 4] = rng.uniform(0.0, 5000.0, n)
    th[:, 5] = rng.uniform(0.0, 5000.0, n)
    th[:, 6] = 100.0
    th[:, 7] = 0.0
    th[:, 8] = 0.0
    th[:, 9] = rng.uniform(0.0, np.pi, n)
    th[:, 10] = 0.3
    th[:, 11] = 1.1
    th[:, 12] = 0.4
    return th


def component_to_chirp(m1, m2):
    """(m1, m2) -> (Mc, q) with q = m2/m1.  Pure unit bookkeeping used to state
    the injections of the workloads in the parameterisation above."""
    mtot = m1 + m2
    eta = m1 * m2 / mtot ** 2
    return mtot * eta ** 0.6, m2 / m1
