"""Writes the lowest eigenvalues of the dense chi_bar0 of a small workload (oracle only).

chi_bar0 = v^{1/2} chi0 v^{1/2} in its dense sum-over-states form on the density
sphere (oracle/pdep.py), from the dense diagonalisation of H in the sphere basis
(every conduction state).  The GPU parity test of the device Davidson compares
its eigenvalues with this file.

    python tests/golden/make_chibar0_golden.py cfg1 32 > tests/golden/chibar0_cfg1.txt
"""
import os
import sys

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import pdep  # noqa: E402


def main():
    name, nlow = sys.argv[1], int(sys.argv[2])
    cfg = workloads.get_config(name)
    s = oracle.build_system(name)
    w, U = np.linalg.eigh(oracle.dense_H(s))
    lam = pdep.chibar0_eigenvalues(s, w, np.ascontiguousarray(U.T), cfg.nv, nlow)
    print(f"# lowest {nlow} eigenvalues of chi_bar0 = v^(1/2) chi0 v^(1/2), {name} "
          f"({cfg.nv} valence bands of {s.npw} plane waves, density sphere "
          f"{len(pdep.density_sphere(s))} points without G = 0, f_s = 2)")
    print("# written by tests/golden/make_chibar0_golden.py (oracle: dense sum over states)")
    for x in lam:
        print(f"{x:.15e}")


if __name__ == "__main__":
    main()
