"""CPU FP64 oracle for the batched Sternheimer hot path.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP library and imports nothing from
the product package; its only inputs are the seeded generators in
``workloads/`` (which hold none of the method's arithmetic) and arrays the
caller passes in.

What it computes (paper: Section 3, the Sternheimer equation and the density
response equation; Section 4.1 for the dual-space Hamiltonian):

  * H = T + V_loc + V_NL on the wave-function sphere, both as a dense matrix
    (plain definition, tiny systems) and by the dual-space FFT route.
  * valence pairs (psi_v, eps_v) by dense diagonalisation or a plain block
    Davidson iteration.
  * Delta psi_jv solving P_c (H - eps_v) P_c x = -P_c Delta V_j psi_v, by a
    dense LU solve, by the sum over all conduction states, or by FP64
    preconditioned conjugate gradient.
  * Delta n_j(r) = f_s sum_v 2 Re[psi_v^*(r) Delta psi_jv(r)] and the chi0
    block Rayleigh-Ritz eigenvalues.

Every function is pinned in ``tests/test_oracle_*.py`` by something other than
itself (closed forms, finite differences, textbook identities); see the
docstrings of those tests.
"""
from .system import System, build_system, build_free_electron_system
from .hamiltonian import dense_H, apply_H, kinetic, to_grid, from_grid, dense_potential_matrix
from .valence import dense_valence, davidson_valence, lobpcg_valence
from .response import (rhs, solve_lu, solve_sum_over_states, tpa_precond, pcg_solve,
                       drho, chi0_block, density, free_electron_response)

__all__ = ["System", "build_system", "build_free_electron_system", "dense_H", "apply_H", "kinetic",
           "to_grid", "from_grid", "dense_potential_matrix", "dense_valence", "davidson_valence", "lobpcg_valence",
           "rhs", "solve_lu", "solve_sum_over_states", "tpa_precond", "pcg_solve", "drho",
           "chi0_block", "density", "free_electron_response"]
