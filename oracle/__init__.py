"""Test oracle (test infrastructure only): plain FP64 CPU reference of the hot path.

Only tests, the smoke check and the benchmark's CPU-baseline leg import this package.
"""
from .core import *  # noqa: F401,F403
from .hmc import covariance_factor, hmc_chain, leapfrog, nuts_chain, nuts_draws_per_sample, nuts_transition  # noqa: F401
from .hmc import dual_averaging, nuts_warmup, nuts_warmup_core  # noqa: F401
