"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds problem parameters and input fields only: initial states,
source terms, tracking targets and perturbation directions, each drawn from a
fixed seed.  It contains none of the solver's arithmetic (no operators, no time
symbols, no transforms), so both the CPU oracle and the GPU path may consume it
without sharing any method code.
"""

from .configs import CONFIGS, Config, get_config, small_config  # noqa: F401
from .fields import (  # noqa: F401
    initial_state,
    initial_velocity,
    source_term,
    source_term_torch,
    source_factors,
    tracking_target,
    fd_directions,
    random_vector,
    hybrid_wave_data,
    hybrid_wave_exact,
    oc_example_data,
    oc_example_exact,
    parareal_initial,
    nonlinear_initial,
)
