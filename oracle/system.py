"""Oracle-side container of one synthetic system (test infrastructure only).

The arrays come straight from the seeded generators in ``workloads`` (or are
passed in by a test); the oracle adds nothing but the G vectors and the grid
index map it needs for its own FFT route.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import workloads


@dataclasses.dataclass
class System:
    L: float
    N: int
    miller: np.ndarray          # [npw, 3] int, caller order
    vloc_r: np.ndarray          # [N, N, N] real
    beta: np.ndarray            # [nproj, npw] complex
    dij: np.ndarray             # [nproj] real
    spin_factor: float = 2.0

    @property
    def omega(self) -> float:
        return self.L ** 3

    @property
    def npw(self) -> int:
        return len(self.miller)

    @property
    def G(self) -> np.ndarray:
        return (2.0 * np.pi / self.L) * self.miller.astype(np.float64)

    @property
    def grid_index(self):
        """Grid index tuple of each sphere point: m mod N along each axis."""
        m = np.mod(self.miller.astype(np.int64), self.N)
        return (m[:, 0], m[:, 1], m[:, 2])


def build_system(cfg_name: str, **overrides) -> System:
    cfg = workloads.get_config(cfg_name, **overrides)
    miller = workloads.miller_sphere(cfg.M2)
    return System(L=cfg.L, N=cfg.N, miller=miller, vloc_r=workloads.vloc_r(cfg),
                  beta=workloads.beta_projectors(cfg, miller), dij=workloads.dij(cfg))


def build_free_electron_system(cfg_name: str) -> System:
    """Same basis and grid as ``cfg_name`` with V_loc = 0 and no projectors."""
    cfg = workloads.get_config(cfg_name)
    miller = workloads.miller_sphere(cfg.M2)
    return System(L=cfg.L, N=cfg.N, miller=miller, vloc_r=np.zeros((cfg.N,) * 3),
                  beta=np.zeros((0, len(miller)), complex), dij=np.zeros(0))
