"""Seeded synthetic workloads for butterfly filtering.

This package generates inputs only: series, time-randomised controls, serving traces and
the bank parameters of each workload.  It holds none of the search arithmetic (no
templates, correlations, norms or reductions), so the GPU library and the CPU oracle can
both consume its output without sharing any code with each other.
"""

from .series import (  # noqa: F401
    chirp_samples,
    white_noise,
    kolmogorov_light_curve,
    time_randomised,
)
from .workloads import (  # noqa: F401
    BankParams,
    WORKLOADS,
    bank_params,
    small_strain_series,
    strain_series,
    light_curve_series,
    light_curve_batch,
    serving_trace,
    serving_segment,
)
