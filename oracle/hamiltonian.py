"""Kohn-Sham Hamiltonian on the plane-wave sphere (oracle; test infrastructure only).

Paper, Section 4.1: the kinetic term acts in reciprocal space, the local
potential in real space (dual-space technique, one inverse and one forward FFT
per application), and only Fourier components inside the kinetic-energy
cutoff sphere are kept.  Section 3 (norm-conserving pseudopotentials) gives
the nonlocal part, here in Kleinman-Bylander form V_NL = sum_p |beta_p> D_p <beta_p|.

FFT conventions: a sphere vector c(G) is placed at grid index m mod N and
taken to real space WITHOUT normalisation, f(r) = sum_G c(G) exp(i G.r); the
forward transform is (1/N^3) sum_r f(r) exp(-i G.r).  The factor
Omega^{-1/2} of psi(r) cancels in H psi.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .system import System

_WORKERS = -1


def kinetic(sys: System) -> np.ndarray:
    """T(G) = |G|^2 / 2 (Hartree)."""
    G = sys.G
    return 0.5 * (G * G).sum(1)


def to_grid(sys: System, c: np.ndarray) -> np.ndarray:
    """Sphere coefficients [..., npw] -> real-space values f(r) = sum_G c(G) e^{iG.r}."""
    N = sys.N
    c = np.asarray(c)
    lead = c.shape[:-1]
    grid = np.zeros(lead + (N, N, N), complex)
    i0, i1, i2 = sys.grid_index
    grid[..., i0, i1, i2] = c
    return scipy.fft.ifftn(grid, axes=(-3, -2, -1), norm="forward", workers=_WORKERS)


def from_grid(sys: System, f: np.ndarray) -> np.ndarray:
    """Real-space values [..., N, N, N] -> sphere coefficients (1/N^3) sum_r f e^{-iG.r}."""
    F = scipy.fft.fftn(f, axes=(-3, -2, -1), norm="forward", workers=_WORKERS)
    i0, i1, i2 = sys.grid_index
    return F[..., i0, i1, i2]


def potential_fourier(sys: System, v_r: np.ndarray) -> np.ndarray:
    """Fourier coefficients V(G) = (1/N^3) sum_r V(r) e^{-iG.r} on the whole grid."""
    return scipy.fft.fftn(v_r, norm="forward", workers=_WORKERS)


def dense_potential_matrix(sys: System, v_r: np.ndarray) -> np.ndarray:
    """Matrix of a local potential in the sphere basis: <G|V|G'> = V(G - G').
    Exact on the sphere when V is band-limited to |m|^2 <= 4 M2 and the grid is
    alias-free (4 max|m_i| + 1 <= N)."""
    VG = potential_fourier(sys, v_r)
    m = sys.miller.astype(np.int64)
    d = m[:, None, :] - m[None, :, :]
    N = sys.N
    return VG[np.mod(d[..., 0], N), np.mod(d[..., 1], N), np.mod(d[..., 2], N)]


def dense_H(sys: System) -> np.ndarray:
    """Plain definition: H(G,G') = |G|^2/2 delta + V_loc(G-G') + sum_p beta_p(G) D_p beta_p(G')^*."""
    H = dense_potential_matrix(sys, sys.vloc_r)
    H[np.diag_indices(sys.npw)] += kinetic(sys)
    if len(sys.dij):
        H += (sys.beta.T * sys.dij) @ sys.beta.conj()
    return H


def apply_local(sys: System, v_r: np.ndarray, c: np.ndarray) -> np.ndarray:
    """(V c)(G) by the dual-space route: inverse FFT, multiply by V(r), forward FFT."""
    return from_grid(sys, v_r * to_grid(sys, c))


def apply_H(sys: System, c: np.ndarray) -> np.ndarray:
    """H c for c [npw] or [nb, npw] by the dual-space (FFT) route."""
    c = np.asarray(c, complex)
    out = apply_local(sys, sys.vloc_r, c) + kinetic(sys) * c
    if len(sys.dij):
        proj = c @ sys.beta.conj().T            # <beta_p|c>  [..., nproj]
        out = out + (proj * sys.dij) @ sys.beta
    return out
