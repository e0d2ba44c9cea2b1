"""Oracle Delta psi and Delta n of sampled solves of a large workload (oracle only).

At 144^3 points and 187,511 plane waves one oracle PCG solve takes about a minute,
too long to repeat inside a GPU test.  This script reads the oracle valence
states cached by make_valence_cache.py (lowest `nv` bands), solves the
Sternheimer equation for the lowest band and perturbations j = 0, 1 with the
oracle's PCG to a true relative residual of 1e-12, and caches Delta psi and
Delta n (Section 3, the linear-response equation and the density response) under
tests/_cache/ (not committed; regenerate with this script).

    python tests/golden/make_response_cache.py cfg5 1
"""
import os
import sys
import time

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), "..", ".."))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402
from make_valence_cache import CACHE, cache_path  # noqa: E402

NPERT = 2


def response_path(name: str, nv: int) -> str:
    cfg = workloads.get_config(name)
    return os.path.join(CACHE, f"{name}_seed{cfg.seed_kb}_nv{nv}_response.npz")


def main():
    name, nv = sys.argv[1], int(sys.argv[2])
    cfg = workloads.get_config(name)
    d = np.load(cache_path(name, nv))
    eps, psi = d["eps"][:nv], d["psi"][:nv]
    s = oracle.build_system(name)
    xs, dns, its = [], [], []
    t0 = time.time()
    for j in range(NPERT):
        dv = workloads.dv_r(cfg, j)
        b = oracle.rhs(s, psi, 0, dv)
        x, it, res, st = oracle.pcg_solve(s, psi, eps, 0, b, tol=1e-12)
        assert st == 0, f"oracle PCG did not converge (perturbation {j})"
        xs.append(x)
        its.append(it)
        dpsi = np.zeros((nv, s.npw), complex)
        dpsi[0] = x
        dns.append(oracle.drho(s, psi, dpsi))
        print(f"{name} j={j}: {it} iterations, residual {res:.2e}, {time.time() - t0:.0f} s",
              flush=True)
    np.savez(response_path(name, nv), dpsi=np.array(xs), drho=np.array(dns), iters=np.array(its),
             band=0)
    print(f"-> {response_path(name, nv)}")


if __name__ == "__main__":
    main()
