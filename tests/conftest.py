import os
import sys

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def cfg1_system():
    import oracle
    return oracle.build_system("cfg1")


@pytest.fixture(scope="session")
def cfg1_dense(cfg1_system):
    """Dense H of config 1 and its full eigendecomposition (rows = eigenvectors)."""
    import numpy as np
    import oracle
    H = oracle.dense_H(cfg1_system)
    w, V = np.linalg.eigh(H)
    return H, w, np.ascontiguousarray(V.T)


@pytest.fixture(scope="session")
def oracle_systems():
    """Oracle systems by name, each built once per session (the 144^3 one, with
    its 2048 projectors over 187,511 plane waves, takes about a minute)."""
    import functools
    import oracle
    return functools.lru_cache(maxsize=3)(oracle.build_system)
