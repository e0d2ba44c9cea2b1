"""Real-in-real-space (Gamma-point) valence states for tests: a basis of the
occupied space whose vectors satisfy c(-G) = conj c(G), by symmetrising the
given states and a Rayleigh-Ritz step on the symmetric basis."""
import numpy as np


def mirror_index(miller):
    """Index of -G for every G of the sphere (caller order)."""
    pos = {tuple(m): i for i, m in enumerate(np.asarray(miller).tolist())}
    return np.array([pos[(-a, -b, -c)] for a, b, c in np.asarray(miller).tolist()])


def realify(psi, miller, apply_h):
    """(eps, psi_sym): Ritz pairs of H on the span of psi, every vector
    c(-G) = conj c(G).  The occupied space of a real Hamiltonian is closed under
    c -> conj c(-G), so the symmetric and antisymmetric parts of its vectors
    span it; the nv largest eigenvalues of their (real) Gram matrix pick an
    orthonormal symmetric basis, and H's (real) matrix in it the rotation."""
    nv = psi.shape[0]
    mir = mirror_index(miller)
    jpsi = psi[:, mir].conj()
    S = np.concatenate([(psi + jpsi) / 2, (psi - jpsi) / 2j])
    G = (S.conj() @ S.T).real
    w, U = np.linalg.eigh((G + G.T) / 2)
    idx = np.argsort(w)[::-1][:nv]
    B = (U[:, idx].T @ S) / np.sqrt(w[idx])[:, None]
    HB = apply_h(B)
    Hs = (B.conj() @ HB.T).real
    e, V = np.linalg.eigh((Hs + Hs.T) / 2)
    return e, np.ascontiguousarray(V.T @ B)
