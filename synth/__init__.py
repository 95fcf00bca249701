"""Seeded synthetic inputs shaped like a DF-MP2 calculation.

This package is the only code shared by the oracle and by the GPU path's
callers (tests, bench).  It draws random numbers and assembles input arrays;
it contains none of the CP-ALS arithmetic of the method itself.
"""
from .generator import (  # noqa: F401
    CONFIGS,
    Config,
    custom_config,
    Inputs,
    make_inputs,
    init_factors,
    planted_factors,
    perturbation,
    amplitude_sequence,
    rank1_t2,
    make_singles,
    rank1_singles,
    exchange_integrals,
    ccd_scale,
)
