"""Computes oracle valence states of a workload and caches them (oracle only).

The full-size GPU parity tests compare Delta psi against the oracle's PCG for
sampled (perturbation, band) pairs; both sides must use the same psi_v, and
the oracle's block LOBPCG takes minutes at these sizes, so its result is
cached under tests/_cache/ (not committed; regenerate with this script).

    python tests/golden/make_valence_cache.py cfg2 [tol] [nv]

A band count `nv` below the workload's keeps only the lowest nv valence bands
(cache file ..._nv{nv}_valence.npz): the parity tests of the 144^3 grid solve
for the lowest band only, which keeps the oracle's eigensolve short.
"""
import os
import sys
import time

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), "..", ".."))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

CACHE = os.path.join(ROOT, "tests", "_cache")


def cache_path(name: str, nv: int = 0) -> str:
    cfg = workloads.get_config(name)
    tag = f"_nv{nv}" if nv and nv != cfg.nv else ""
    return os.path.join(CACHE, f"{name}_seed{cfg.seed_kb}{tag}_valence.npz")


def main():
    name = sys.argv[1]
    tol = float(sys.argv[2]) if len(sys.argv) > 2 else 1e-11
    nv = int(sys.argv[3]) if len(sys.argv) > 3 else 0
    cfg = workloads.get_config(name)
    if nv:
        cfg = workloads.get_config(name, nv=nv)
    s = oracle.build_system(name)
    t0 = time.time()
    nb = cfg.nv + 8
    eps, psi, res, it = oracle.lobpcg_valence(s, nb, tol=tol, nconv=cfg.nv + 1, verbose=True)
    os.makedirs(CACHE, exist_ok=True)
    np.savez(cache_path(name, nv), eps=eps, psi=psi, res=res, iters=it, tol=tol)
    print(f"{name}: {nb} bands, residual {res:.2e}, {it} iterations, {time.time() - t0:.0f} s, "
          f"gap {eps[cfg.nv] - eps[cfg.nv - 1]:.6f} Ha -> {cache_path(name, nv)}")


if __name__ == "__main__":
    main()
