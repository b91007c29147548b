"""Seeded synthetic workloads shared by the GPU library's tests/bench and the oracle.

This package only builds inputs: grids, boundary flags, Lame fields, sponge
profiles, source and receiver lists. It holds none of the scheme's arithmetic,
so the oracle and the GPU path can both read the same problem description
without sharing any of the method's code.
"""
from .problem import (BC_FREE, BC_FREE0, BC_PERIODIC, BC_RIGID, Medium, Problem, Source,
                      default_sponge_profile, ring_receivers)
from .configs import (plain_small, plain_large, hbm_scale, batched_shots,
                      adjoint_shots, CONFIG_NAMES)

__all__ = [
    "BC_FREE", "BC_FREE0", "BC_PERIODIC", "BC_RIGID", "Medium", "Problem", "Source",
    "default_sponge_profile", "ring_receivers", "plain_small", "plain_large",
    "hbm_scale", "batched_shots", "adjoint_shots", "CONFIG_NAMES",
]
