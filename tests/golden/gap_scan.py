"""Scan KB-coefficient seeds for a gap above the last valence band (oracle only).

For each seed the oracle's LOBPCG finds the lowest nv + 8 eigenvalues of the
synthetic Hamiltonian to a loose residual and reports eps[nv] - eps[nv-1].  The
first seed with a gap >= 0.05 Ha is the one the workload uses.  Writes one line
per seed to stdout:  config seed D_s D_p gap_Ha eps_nv-1 eps_nv residual.

    python tests/golden/gap_scan.py cfg2 0 1 2 3 ...
"""
import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    name = sys.argv[1]
    tol = float(os.environ.get("GAP_TOL", "1e-4"))
    for seed in map(int, sys.argv[2:]):
        cfg = workloads.get_config(name, seed_kb=seed)
        s = oracle.build_system(name, seed_kb=seed)
        nb = cfg.nv + 8
        if s.npw <= 4000:
            w, _ = oracle.dense_valence(s, nb)
            res = 0.0
        else:
            w, _, res, _ = oracle.lobpcg_valence(s, nb, tol=tol, nconv=cfg.nv + 1)
        d = workloads.dij(cfg)
        ds, dp = d[0], (d[1] if cfg.channels == 4 else float("nan"))
        print(f"{name} {seed} {ds:+.4f} {dp:+.4f} {w[cfg.nv] - w[cfg.nv - 1]:.6f} "
              f"{w[cfg.nv - 1]:.6f} {w[cfg.nv]:.6f} {res:.1e}", flush=True)


if __name__ == "__main__":
    main()
