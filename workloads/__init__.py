"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*: the plane-wave basis (Miller indices of
the wave-function sphere), the synthetic crystal's local potential on the real
space grid, Kleinman-Bylander projectors, their coefficients and the random
smooth perturbations Delta V_j.  It contains none of the Sternheimer method's
arithmetic (no Hamiltonian application, no projection, no solve, no density
response); those live separately in ``oracle/`` (CPU reference) and in the HIP
library.
"""
from .crystal import (CONFIGS, Config, get_config, miller_sphere, vloc_r, beta_projectors,
                      dij, dv_r, dv_block, atom_positions, grid_gvectors)

__all__ = ["CONFIGS", "Config", "get_config", "miller_sphere", "vloc_r", "beta_projectors",
           "dij", "dv_r", "dv_block", "atom_positions", "grid_gvectors"]
