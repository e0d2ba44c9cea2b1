"""CPU checks of the Gamma-point state preparation used by the GPU tests
(tests/gamma_util.py): on the config-1 crystal its output must be real in real
space, orthonormal, eigenstates of the dense H with the dense eigenvalues, and
span the same occupied space as the given states.  A real-space check ties
the symmetry to its meaning: the grid values of a symmetric state are real.
Also pins the half-sphere identity the Gamma-point products rest on, with the
oracle's own H: for symmetric a and b, <a, b> = 2 Re sum over the half from
G = 0 on minus the G = 0 term, in any order that puts -G before G = 0 for
every G after it."""
import numpy as np

import gamma_util
import oracle


def test_realify_gives_symmetric_eigenstates(cfg1_system, cfg1_dense):
    s = cfg1_system
    H, w, V = cfg1_dense
    nv = 8
    # the dense eigenvectors carry arbitrary phases, so they are not symmetric
    mir = gamma_util.mirror_index(s.miller)
    assert np.abs(V[:nv, mir].conj() - V[:nv]).max() > 1e-3
    eps, psi = gamma_util.realify(V[:nv], s.miller, lambda B: (H @ B.T).T)
    assert np.abs(psi[:, mir].conj() - psi).max() < 1e-13
    assert np.abs(psi.conj() @ psi.T - np.eye(nv)).max() < 1e-13
    assert np.abs(eps - w[:nv]).max() < 1e-12
    R = (H @ psi.T).T - eps[:, None] * psi
    assert np.abs(R).max() < 1e-12
    P_in = V[:nv].T @ V[:nv].conj()
    P_out = psi.T @ psi.conj()
    assert np.abs(P_in - P_out).max() < 1e-12
    # real in real space: the grid values of a symmetric state are real, those
    # of the given (phase-rotated) states are not
    grid = oracle.to_grid(s, psi)
    assert np.abs(grid.imag).max() < 1e-13 * np.abs(grid.real).max()
    g0 = oracle.to_grid(s, V[:nv])
    assert np.abs(g0.imag).max() > 1e-3 * np.abs(g0).max()


def test_half_sphere_identity(cfg1_system, cfg1_dense):
    s = cfg1_system
    H, w, V = cfg1_dense
    eps, psi = gamma_util.realify(V[:8], s.miller, lambda B: (H @ B.T).T)
    a = psi[3]
    b = oracle.apply_H(s, psi[5][None])[0] + 0.3 * psi[1]   # symmetric: H is real
    m = np.asarray(s.miller)
    # an order with every -G of the second half before G = 0: sort by the
    # first nonzero Miller index's sign, G = 0 in the middle
    key = np.array([np.sign(x[np.flatnonzero(x)[0]]) if np.any(x) else 0 for x in m])
    order = np.argsort(key, kind="stable")
    k0 = int(np.flatnonzero(key[order] == 0)[0])
    ao, bo = a[order], b[order]
    full = np.vdot(a, b)
    half = 2.0 * np.vdot(ao[k0:], bo[k0:]).real - (np.conj(ao[k0]) * bo[k0]).real
    assert abs(full.imag) < 1e-13 * abs(full) + 1e-15
    assert abs(half - full.real) < 1e-13 * max(1.0, abs(full))
