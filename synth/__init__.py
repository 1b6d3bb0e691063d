"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package only *draws* inputs (coordinates, per-atom parameters, topology).
It holds none of the force-field or optimizer arithmetic: both the CPU oracle
and the GPU library receive what it produces and compute from there.
"""
from .chain import (  # noqa: F401
    GENERATOR_VERSION,
    SplitMix64,
    chain_system,
    batch_sizes,
    config_system,
    CONFIGS,
    COULOMB_KCAL,
)
