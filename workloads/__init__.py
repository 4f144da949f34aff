"""Seeded synthetic workloads for the SWR-Galerkin hot path.

This package holds only *inputs*: the physical and numerical parameters of
each workload and the seeded random draws some of them need.  It contains
none of the method's arithmetic (no geometry, no basis, no integrals), so
that both the CPU oracle and the HIP library can read it without sharing
any code path with each other.
"""
from .configs import (  # noqa: F401
    CONFIGS,
    get_config,
    random_small_configs,
    slater_configs,
    lsd_configs,
    lo_configs,
    tiny_configs,
)
