"""Valence eigenpairs (oracle; test infrastructure only).

The paper takes psi_v and eps_v from a ground-state DFT run (Section 3).  For
the synthetic systems they are the lowest eigenpairs of H: by dense
diagonalisation (small bases) or by a plain block Davidson iteration
(Davidson's method, which the paper uses for the dielectric matrix in
Section 3, applied here to H itself).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import dense_H, apply_H, kinetic
from .system import System


def _orth_against(V, HV, Q, HQ, drop=1e-10):
    """Remove from the rows of V (and consistently from HV) their components along the
    orthonormal rows of Q, then orthonormalise V; done twice for stability.  Directions
    whose squared norm falls below ``drop`` (relative) are dropped, which bounds the
    error amplification of the implicitly updated HV.  Returns (V', HV')."""
    nrm = np.linalg.norm(V, axis=1)
    nrm[nrm == 0] = 1.0
    V = V / nrm[:, None]
    HV = HV / nrm[:, None] if HV is not None else None
    for _ in range(2):
        if Q is not None and len(Q):
            C = V @ Q.conj().T
            V = V - C @ Q
            HV = HV - C @ HQ if HV is not None else None
        G = V.conj() @ V.T
        G = 0.5 * (G + G.conj().T)
        w, U = np.linalg.eigh(G)
        keep = w > drop * max(w.max(), 1e-300)
        T = U[:, keep] / np.sqrt(w[keep])
        V = T.T @ V
        HV = T.T @ HV if HV is not None else None
    return V, HV


def dense_valence(sys: System, nbands: int):
    """Lowest ``nbands`` eigenpairs of the dense H: (eps [nbands], psi [nbands, npw])."""
    w, V = scipy.linalg.eigh(dense_H(sys), subset_by_index=[0, nbands - 1])
    return w, np.ascontiguousarray(V.T)


def _orthonormalise(V: np.ndarray, against: np.ndarray | None = None) -> np.ndarray:
    """Rows of V made orthonormal (and orthogonal to the rows of ``against``)."""
    for _ in range(2):
        if against is not None and len(against):
            V = V - (V @ against.conj().T) @ against
        q, _ = np.linalg.qr(V.T)
        V = q.T
    return V


def davidson_valence(sys: System, nbands: int, tol: float = 1e-11, maxit: int = 400,
                     seed: int = 7, max_subspace: int = 3, verbose: bool = False):
    """Block Davidson for the lowest ``nbands`` eigenpairs of H (FFT route).

    Subspace V (orthonormal rows); each iteration: Rayleigh-Ritz on V, residuals
    R = H x - theta x of the Ritz vectors, diagonal correction
    t = R / (max(T(G) - theta, 0) + 1) filtered against V, appended; restart from the
    current Ritz vectors when V exceeds ``max_subspace * nbands``.  Converged
    when every residual norm ||R_i|| <= tol.
    """
    rng = np.random.default_rng(seed)
    npw = sys.npw
    T = kinetic(sys)
    # start from low-kinetic-energy random vectors
    X = (rng.standard_normal((nbands, npw)) + 1j * rng.standard_normal((nbands, npw)))
    X /= (1.0 + T)[None, :] ** 2
    V = _orthonormalise(X)
    HV = apply_H(sys, V)
    res = np.inf
    for it in range(maxit):
        Hs = V.conj() @ HV.T
        Hs = 0.5 * (Hs + Hs.conj().T)
        theta, Y = scipy.linalg.eigh(Hs)
        theta, Y = theta[:nbands], Y[:, :nbands]
        X = Y.T @ V
        HX = Y.T @ HV
        R = HX - theta[:, None] * X
        rn = np.linalg.norm(R, axis=1)
        res = rn.max()
        if verbose:
            print(f"davidson it {it} dim {len(V)} max|R| {res:.3e}", flush=True)
        if res <= tol:
            return theta, X, res, it
        act = rn > tol
        t = R[act] / (np.maximum(T[None, :] - theta[act, None], 0.0) + 1.0)
        if len(V) + act.sum() > max_subspace * nbands:
            V, HV = X, HX      # Ritz vectors are orthonormal: restart on them
        t = _orthonormalise(t, against=V)
        V = np.vstack([V, t])
        HV = np.vstack([HV, apply_H(sys, t)])
    raise RuntimeError(f"oracle Davidson did not converge: max residual {res:.3e}")


def lobpcg_valence(sys: System, nbands: int, tol: float = 1e-11, maxit: int = 500,
                   seed: int = 7, nconv: int | None = None, verbose: bool = False):
    """Locally optimal block preconditioned conjugate gradient (Knyazev) for the lowest
    ``nbands`` eigenpairs of H by the FFT route.  Each iteration: residuals
    R = H X - X theta, preconditioned W = R / (max(T - theta, 0) + 1), Rayleigh-Ritz on
    span[X, W, P] (P = previous update), keep the lowest ``nbands``.  Converged when the
    residual norms of the lowest ``nconv`` (default all) Ritz pairs are <= tol.
    Returns (theta [nbands], X [nbands, npw], max residual, iterations)."""
    rng = np.random.default_rng(seed)
    npw = sys.npw
    T = kinetic(sys)
    nconv = nbands if nconv is None else nconv
    X = (rng.standard_normal((nbands, npw)) + 1j * rng.standard_normal((nbands, npw)))
    X /= (1.0 + T)[None, :] ** 2
    X, _ = _orth_against(X, None, None, None)
    HX = apply_H(sys, X)
    P = HP = None
    res = np.inf
    for it in range(maxit):
        if it % 8 == 0:
            HX = apply_H(sys, X)                     # refresh the implicitly updated products
        X, HX = _orth_against(X, HX, None, None)   # keep X orthonormal (HX transformed alike)
        Hs = X.conj() @ HX.T
        theta, Y = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T))
        X, HX = Y.T @ X, Y.T @ HX
        R = HX - theta[:, None] * X
        rn = np.linalg.norm(R, axis=1)
        res = rn[:nconv].max()
        if verbose:
            print(f"lobpcg it {it} max|R| {res:.3e}", flush=True)
        if res <= tol:
            return theta, X, res, it
        W = R / (np.maximum(T[None, :] - theta[:, None], 0.0) + 1.0)
        W, _ = _orth_against(W, None, X, HX)
        HW = apply_H(sys, W)
        S, HS = np.vstack([X, W]), np.vstack([HX, HW])
        if P is not None:
            P, _ = _orth_against(P, None, S, None)
            HP = apply_H(sys, P)                     # explicit: P may be nearly dependent
            S, HS = np.vstack([S, P]), np.vstack([HS, HP])
        Hs = S.conj() @ HS.T
        Gs = S.conj() @ S.T
        w, C = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T), 0.5 * (Gs + Gs.conj().T))
        C = C[:, :nbands]
        X, HX = C.T @ S, C.T @ HS
        # new search direction from the W and P parts only (no cancellation against X)
        P, HP = C[nbands:].T @ S[nbands:], C[nbands:].T @ HS[nbands:]
    raise RuntimeError(f"oracle LOBPCG did not converge: max residual {res:.3e}")
