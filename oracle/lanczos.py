"""Lanczos chains of the frequency-dependent response (oracle; test infrastructure only).

Paper, Section 3 (equation "lanczos" and the recurrences before it): for an
orbital psi_i and a real function phi_m (a PDEP vector), the chain starts from
|psi_i phi_m> and runs the three-term recurrence of H,
    beta^{l+1} q^{l+1} = (H - alpha^l) q^l - beta^l q^{l-1},
    alpha^l = <q^l|H|q^l>,  q^0 = 0,
each new vector also orthogonalised against every earlier vector of its chain
(one classical Gram-Schmidt pass after the three-term step).  The tridiagonal
matrix of the alpha (diagonal) and beta (off-diagonal) has eigenvalues d and
eigenvectors U; the braket <u_n | q^l_m> of the start vectors with the chain
vectors completes the frequency dependence (Section 4.3 computes it as one
matrix product).  Conventions: u_m = T_S[phi_m psi_i] on the sphere (the
product taken in real space, FFT route), beta^1 = ||u_m||, q^1 = u_m / beta^1.
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_H, apply_local
from .system import System


def start_vectors(sys: System, psi_i: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """u_m = T_S[phi_m psi_i] for real grids phi [nm, N, N, N]: [nm, npw]."""
    return np.stack([apply_local(sys, phi[m], psi_i) for m in range(len(phi))])


def lanczos_chain(sys: System, u: np.ndarray, nsteps: int):
    """One chain from the start vector u: (alpha [nsteps], beta [nsteps], Q [nsteps, npw]).
    beta[0] = ||u||; beta[l] (l >= 1) is the norm that made q^{l+1}, the off-diagonal
    T[l-1, l] of the tridiagonal matrix."""
    beta = [np.linalg.norm(u)]
    Q = [u / beta[0]]
    alpha = []
    for l in range(nsteps):
        hq = apply_H(sys, Q[l])
        a = float(np.real(np.vdot(Q[l], hq)))
        alpha.append(a)
        r = hq - a * Q[l]
        if l > 0:
            r = r - beta[l] * Q[l - 1]
        c = np.array([np.vdot(Q[k], r) for k in range(l + 1)])
        r = r - c @ np.array(Q[:l + 1])
        if l < nsteps - 1:
            b = np.linalg.norm(r)
            beta.append(b)
            Q.append(r / b)
    return np.array(alpha), np.array(beta), np.array(Q)


def tridiagonal(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """The Lanczos matrix: alpha on the diagonal, beta[1:] beside it."""
    T = np.diag(alpha)
    off = beta[1:len(alpha)]
    T[np.arange(len(off)), np.arange(1, len(off) + 1)] = off
    T[np.arange(1, len(off) + 1), np.arange(len(off))] = off
    return T


def lanczos_block(sys: System, psi_i: np.ndarray, phi: np.ndarray, nsteps: int):
    """Every chain of one orbital: alpha, beta [nm, L], d [nm, L] ascending,
    U [nm, L, L] (columns = eigenvectors), braket [nm, nm, L] = <u_n | q^l_m>."""
    u = start_vectors(sys, psi_i, phi)
    nm = len(u)
    A = np.empty((nm, nsteps))
    B = np.empty((nm, nsteps))
    D = np.empty((nm, nsteps))
    U = np.empty((nm, nsteps, nsteps))
    Qs = []
    for m in range(nm):
        a, b, Q = lanczos_chain(sys, u[m], nsteps)
        A[m], B[m] = a, b
        D[m], U[m] = np.linalg.eigh(tridiagonal(a, b))
        Qs.append(Q)
    braket = np.einsum("ng,mlg->nml", u.conj(), np.array(Qs))
    return A, B, D, U, braket
