"""Oracle responses of large workloads, stored for the GPU parity tests (oracle only).

Reads the oracle valence states stored by make_valence_cache.py and solves the
Sternheimer equation (Section 3, the linear-response equation) with the
oracle's FP64 PCG to a true relative residual of 1e-12, then forms the density
responses (Section 3, the density-response equation) and the chi0 block
Rayleigh-Ritz.  Output under tests/oracle_data/ (compressed npz, committed).

    python tests/golden/make_response_cache.py cfg2        # 2 perturbations x all 128 bands
    python tests/golden/make_response_cache.py cfg5 1      # lowest band, 2 perturbations

cfg2: Delta n_0, Delta n_1, the chi0 block (M, S, eigenvalues) and four sampled
Delta psi; the 256 solves run in a process pool of single-threaded workers.
cfg5 (one band): Delta psi of perturbations 0 and 1 only (Delta n of one band
is a cheap oracle product the test forms itself).
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
from make_valence_cache import DATA, cache_path  # noqa: E402

NPERT = 2
SAMPLES = [(0, 0), (0, 127), (1, 64), (1, 100)]


def response_path(name: str, nv: int = 0) -> str:
    cfg = workloads.get_config(name)
    tag = f"_nv{nv}" if nv and nv != cfg.nv else ""
    return os.path.join(DATA, f"{name}_seed{cfg.seed_kb}{tag}_response.npz")


_W = {}


def _init(name, nv):
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle.hamiltonian as oh
    oh._WORKERS = 1
    d = np.load(cache_path(name, nv))
    _W["s"] = oracle.build_system(name)
    _W["eps"], _W["psi"] = d["eps"][:nv], d["psi"][:nv]
    _W["cfg"] = workloads.get_config(name)


def _solve(jv):
    j, v = jv
    s, eps, psi = _W["s"], _W["eps"], _W["psi"]
    b = oracle.rhs(s, psi, v, workloads.dv_r(_W["cfg"], j))
    x, it, res, st = oracle.pcg_solve(s, psi, eps, v, b, tol=1e-12)
    assert st == 0, f"oracle PCG did not converge (perturbation {j}, band {v})"
    return j, v, x, it


def main():
    name = sys.argv[1]
    cfg = workloads.get_config(name)
    nv = int(sys.argv[2]) if len(sys.argv) > 2 else cfg.nv
    t0 = time.time()
    if nv == 1:
        _init(name, nv)
        xs, its = [], []
        for j in range(NPERT):
            _, _, x, it = _solve((j, 0))
            xs.append(x)
            its.append(it)
            print(f"{name} j={j}: {it} iterations, {time.time() - t0:.0f} s", flush=True)
        np.savez_compressed(response_path(name, nv), dpsi=np.array(xs), iters=np.array(its),
                            band=0)
    else:
        import multiprocessing as mp
        pairs = [(j, v) for j in range(NPERT) for v in range(nv)]
        dpsi = {}
        its = np.zeros((NPERT, nv), int)
        with mp.get_context("fork").Pool(os.cpu_count(), _init, (name, nv)) as pool:
            for k, (j, v, x, it) in enumerate(pool.imap_unordered(_solve, pairs, chunksize=4)):
                dpsi[(j, v)] = x
                its[j, v] = it
                if (k + 1) % 32 == 0:
                    print(f"{k + 1} of {len(pairs)} solves, {time.time() - t0:.0f} s", flush=True)
        d = np.load(cache_path(name, nv))
        s = oracle.build_system(name)
        psi = d["psi"][:nv]
        dn = np.stack([oracle.drho(s, psi, np.stack([dpsi[(j, v)] for v in range(nv)]))
                       for j in range(NPERT)])
        dv = workloads.dv_block(cfg, range(NPERT))
        lam, M, S = oracle.chi0_block(s, dv, dn)
        np.savez_compressed(response_path(name), drho=dn, M=M, S=S, lam=lam, iters=its,
                            samples=np.array(SAMPLES),
                            dpsi_samples=np.stack([dpsi[jv] for jv in SAMPLES]))
    print(f"-> {response_path(name, nv)} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
