"""Computes oracle valence states of a workload and stores them (oracle only).

The full-size GPU parity tests compare against the oracle on systems whose
valence states take the oracle's block LOBPCG minutes to an hour; both sides
must use the same psi_v, so the oracle's result is stored under
tests/oracle_data/ (compressed npz, committed) and read by the tests.

    python tests/golden/make_valence_cache.py cfg2 [tol] [nv]

The file holds the lowest nv + 1 eigenpairs (the extra one gives the gap) of
the nv + 8 the LOBPCG iterates.  A band count `nv` below the workload's keeps
only the lowest nv valence bands (file ..._nv{nv}_valence.npz).
"""
import os
import sys
import time

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), "..", ".."))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

DATA = os.path.join(ROOT, "tests", "oracle_data")


def cache_path(name: str, nv: int = 0) -> str:
    cfg = workloads.get_config(name)
    tag = f"_nv{nv}" if nv and nv != cfg.nv else ""
    return os.path.join(DATA, f"{name}_seed{cfg.seed_kb}{tag}_valence.npz")


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
    os.makedirs(DATA, exist_ok=True)
    keep = cfg.nv + 1
    np.savez_compressed(cache_path(name, nv), eps=eps[:keep], psi=psi[:keep], res=res, iters=it,
                        tol=tol)
    print(f"{name}: {nb} bands, residual {res:.2e}, {it} iterations, {time.time() - t0:.0f} s, "
          f"gap {eps[cfg.nv] - eps[cfg.nv - 1]:.6f} Ha -> {cache_path(name, nv)}")


if __name__ == "__main__":
    main()
