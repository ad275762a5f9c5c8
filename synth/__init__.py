"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module builds the *inputs* of the relative-binned likelihood (frequency
grid, PSD, detector geometry, Gaussian noise, parameter draws and the workload
configurations).  It holds none of the likelihood or waveform arithmetic: no
waveform, antenna pattern, inner product or binning is computed here, so sharing
it between the oracle and the GPU path cannot hide a mistake in either.
"""
from .inputs import (  # noqa: F401
    PARAM_NAMES,
    N_PARAMS,
    frequency_grid,
    analytic_psd,
    detector_geometry,
    gaussian_noise,
    draw_theta,
    mismatch_draws,
    PRIORS,
)
from .configs import (  # noqa: F401
    CONFIGS,
    workload,
    N_SERVE_EVENTS,
    SERVE_RATE_HZ,
    serving_event,
    serving_inputs,
    serving_stream,
)
