"""Dielectric eigenpairs in dense form (oracle; test infrastructure only).

Paper, Section 3: the dielectric response enters through the eigenpairs of the
symmetrised irreducible density response chi_bar0 = v^{1/2} chi0 v^{1/2} (v the
bare Coulomb interaction), which the paper's code finds by an iterative
(Davidson) eigensolver that applies chi0 through Sternheimer solves.  The plain
definition written out here: chi0 as the sum over every conduction state of the
sphere basis (the textbook sum-over-states form of the density response; with a
complete conduction manifold it equals what the Sternheimer equation gives),

    Delta n = chi0 Delta V,   Delta n(r) = f_s sum_v [psi_v^*(r) Delta psi_v(r) + c.c.],
    Delta psi_v = sum_c |c> <c|Delta V|v> / (eps_v - eps_c),

as a matrix on the density sphere |m|^2 <= 4 max|m_sphere|^2 (the support of a
product of two sphere functions) without G = 0, in the coefficient convention
f(r) = sum_G f(G) e^{iG.r} for real perturbations Delta V.  v^{1/2}(G) =
sqrt(4 pi) / |G|; chi_bar0(G, G') = v^{1/2}(G) chi0(G, G') v^{1/2}(G').  The
eigenvalues of that matrix are those of chi_bar0 as an operator (the L2 inner
product is Omega sum_G, a constant multiple of the coefficient one).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg

from .hamiltonian import to_grid
from .system import System


def density_sphere(sys: System) -> np.ndarray:
    """Miller indices [nG, 3] of the density sphere without G = 0 (lexicographic order)."""
    m2 = int((sys.miller.astype(np.int64) ** 2).sum(1).max())
    r = int(np.floor(np.sqrt(4 * m2)))
    ax = np.arange(-r, r + 1)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    q = (m * m).sum(1)
    return m[(q <= 4 * m2) & (q > 0)]


def coulomb_sqrt(sys: System, mG: np.ndarray) -> np.ndarray:
    """v^{1/2}(G) = sqrt(4 pi) / |G| for G = (2 pi / L) m."""
    G = (2.0 * np.pi / sys.L) * np.sqrt((mG.astype(np.float64) ** 2).sum(1))
    return np.sqrt(4.0 * np.pi) / G


def chi0_matrix(sys: System, evals: np.ndarray, evecs: np.ndarray, nv: int,
                mG: np.ndarray) -> np.ndarray:
    """chi0(G, G') on the rows mG [nG, 3] from all eigenpairs (evals ascending, evecs
    [nbasis, npw] orthonormal; the first nv are the valence states)."""
    N = sys.N
    idx = tuple(np.mod(mG[:, k].astype(np.int64), N) for k in range(3))
    a = to_grid(sys, evecs[:nv])               # unnormalised: psi = Omega^{-1/2} a
    c = to_grid(sys, evecs[nv:])
    nG = len(mG)
    chi = np.zeros((nG, nG), complex)
    for v in range(nv):
        # pair densities psi_v^* psi_c and psi_c^* psi_v, Fourier coefficients
        # (1/Omega) int rho e^{-iG.r} dr = (1/N^3) sum_r rho e^{-iG.r}
        rho_vc = np.conj(a[v])[None] * c / sys.omega
        f_vc = scipy.fft.fftn(rho_vc, axes=(1, 2, 3), norm="forward")[:, idx[0], idx[1], idx[2]]
        f_cv = scipy.fft.fftn(np.conj(rho_vc), axes=(1, 2, 3), norm="forward")[:, idx[0], idx[1], idx[2]]
        w = 1.0 / (evals[v] - evals[nv:])     # negative: every conduction state lies above
        # <c|Delta V|v> = Omega sum_G' conj(rho_vc(G')) Delta V(G'); its conjugate pairs
        # with the c.c. term through rho_cv
        chi += (f_vc.T * w) @ np.conj(f_vc)
        chi += (f_cv.T * w) @ np.conj(f_cv)
    return sys.spin_factor * sys.omega * chi


def chibar0_matrix(sys: System, evals: np.ndarray, evecs: np.ndarray, nv: int):
    """(mG, chi_bar0 matrix [nG, nG]) on the density sphere without G = 0."""
    mG = density_sphere(sys)
    s = coulomb_sqrt(sys, mG)
    chi = chi0_matrix(sys, evals, evecs, nv, mG)
    return mG, s[:, None] * chi * s[None, :]


def chibar0_eigenvalues(sys: System, evals: np.ndarray, evecs: np.ndarray, nv: int,
                        nlow: int) -> np.ndarray:
    """The nlow lowest (most negative) eigenvalues of chi_bar0, ascending."""
    _, K = chibar0_matrix(sys, evals, evecs, nv)
    K = 0.5 * (K + K.conj().T)
    return scipy.linalg.eigh(K, eigvals_only=True, subset_by_index=[0, nlow - 1])


def apply_matrix_to_real(sys: System, mG: np.ndarray, K: np.ndarray, f_r: np.ndarray) -> np.ndarray:
    """(K f)(r) for a real band-limited grid function f: coefficients of f on mG (f has
    none at G = 0 and outside the sphere), K applied, back to the grid."""
    N = sys.N
    idx = tuple(np.mod(mG[:, k].astype(np.int64), N) for k in range(3))
    F = scipy.fft.fftn(f_r, norm="forward")[idx]
    out = np.zeros((N, N, N), complex)
    out[idx] = K @ F
    return np.real(scipy.fft.ifftn(out, norm="forward"))
