"""Oracle results stored under tests/oracle_data/ (compressed npz, committed).

They are written by tests/golden/make_valence_cache.py and
tests/golden/make_response_cache.py, which call only the oracle: valence
states whose oracle eigensolve takes minutes to an hour, and PCG responses of
the large workloads.  A missing file is an error (the files are committed).
"""
import os

import numpy as np
import pytest

import workloads

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_data")


def _path(name: str, kind: str, nv: int = 0) -> str:
    cfg = workloads.get_config(name)
    tag = f"_nv{nv}" if nv and nv != cfg.nv else ""
    return os.path.join(DATA, f"{name}_seed{cfg.seed_kb}{tag}_{kind}.npz")


def load(name: str, kind: str, nv: int = 0):
    p = _path(name, kind, nv)
    if not os.path.exists(p):
        script = "make_valence_cache.py" if kind == "valence" else "make_response_cache.py"
        pytest.fail(f"oracle data {p} missing: regenerate with tests/golden/{script}")
    return np.load(p)


def valence(name: str, nv: int = 0):
    """(eps, psi) of the lowest nv + 1 bands (nv = the workload's band count by default)."""
    d = load(name, "valence", nv)
    return d["eps"], d["psi"]
