"""Pins of the oracle's valence eigensolvers (CPU only): the iterative solvers
must reproduce dense diagonalisation, and the free-electron closed form."""
import numpy as np

import oracle


def test_lobpcg_and_davidson_match_dense(cfg1_system, cfg1_dense):
    H, w, V = cfg1_dense
    for solver in (oracle.lobpcg_valence, oracle.davidson_valence):
        th, X, res, it = solver(cfg1_system, 12, tol=1e-11)
        assert np.abs(th - w[:12]).max() < 1e-12
        R = X @ H.T - th[:, None] * X
        assert np.linalg.norm(R, axis=1).max() < 1e-10
        assert np.abs(X.conj() @ X.T - np.eye(12)).max() < 1e-12


def test_free_electron_lowest_shells():
    s = oracle.build_free_electron_system("cfg1")
    th, X, res, it = oracle.lobpcg_valence(s, 19, tol=1e-10)
    b = 2 * np.pi / s.L
    expect = 0.5 * b * b * np.array([0] + [1] * 6 + [2] * 12)
    assert np.abs(th - expect).max() < 1e-12


def test_dense_valence_gap(cfg1_system):
    """The config-1 crystal has a gap above band 8 (needed for a nonsingular
    Sternheimer operator on the top valence band)."""
    w, _ = oracle.dense_valence(cfg1_system, 9)
    assert w[8] - w[7] > 0.05
