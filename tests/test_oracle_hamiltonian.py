"""Pins of the oracle's basis, FFT conventions and Hamiltonian (CPU only).

Each check compares the oracle against something it does not compute itself:
closed forms (plane waves, free-electron spectrum with the r_3(n) shell
degeneracies of tests/golden/r3_shells.txt), an independent route (dense
convolution matrix vs the dual-space FFT route of Section 4.1), or an exact
symmetry (Hermiticity, rigid translation of the crystal).
"""
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_plane_wave_maps_to_single_grid_harmonic(cfg1_system):
    """to_grid(e_G0)(r) = exp(i G0.r) at every grid point (sign, placement)."""
    s = cfg1_system
    k = 123
    c = np.zeros(s.npw, complex)
    c[k] = 1.0
    f = oracle.to_grid(s, c)
    N, L = s.N, s.L
    x = np.arange(N) * L / N
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1)
    expect = np.exp(1j * (X @ s.G[k]))
    assert np.abs(f - expect).max() < 1e-12


def test_fft_round_trip_and_parseval(cfg1_system):
    s = cfg1_system
    rng = np.random.default_rng(1)
    c = _rand(rng, 3, s.npw)
    f = oracle.to_grid(s, c)
    assert np.abs(oracle.from_grid(s, f) - c).max() < 1e-13
    # Parseval: (1/N^3) sum_r |f|^2 = sum_G |c|^2
    lhs = (np.abs(f) ** 2).sum(axis=(1, 2, 3)) / s.N ** 3
    assert np.allclose(lhs, (np.abs(c) ** 2).sum(1), rtol=1e-13)


def test_sphere_counts_match_brute_force():
    for name in ("cfg1", "cfg2", "cfg4a"):
        cfg = workloads.get_config(name)
        m = workloads.miller_sphere(cfg.M2)
        r = int(np.sqrt(cfg.M2)) + 1
        cnt = sum(1 for a in range(-r, r + 1) for b in range(-r, r + 1) for c in range(-r, r + 1)
                  if a * a + b * b + c * c <= cfg.M2)
        assert len(m) == cnt
        assert len(np.unique(m, axis=0)) == len(m)
        assert 4 * np.abs(m).max() + 1 <= cfg.N          # alias-free grid


def test_free_electron_spectrum_and_degeneracies():
    """V_loc = 0, no projectors: eigenvalues b^2 n / 2 with multiplicity r_3(n)."""
    s = oracle.build_free_electron_system("cfg1")
    w = np.linalg.eigvalsh(oracle.dense_H(s))
    table = np.loadtxt(os.path.join(GOLDEN, "r3_shells.txt"), dtype=int)
    b = 2 * np.pi / s.L
    levels = np.round(w / (0.5 * b * b)).astype(int)
    assert np.abs(w - 0.5 * b * b * levels).max() < 1e-12
    for n, r3 in table:
        assert (levels == n).sum() == r3, n


def test_dense_and_fft_routes_agree(cfg1_system):
    s = cfg1_system
    H = oracle.dense_H(s)
    rng = np.random.default_rng(2)
    c = _rand(rng, 4, s.npw)
    a = c @ H.T
    b = oracle.apply_H(s, c)
    assert np.abs(a - b).max() / np.abs(a).max() < 1e-13


def test_hermiticity(cfg1_system):
    s = cfg1_system
    H = oracle.dense_H(s)
    assert np.abs(H - H.conj().T).max() < 1e-14
    rng = np.random.default_rng(3)
    a, b = _rand(rng, s.npw), _rand(rng, s.npw)
    lhs = np.vdot(a, oracle.apply_H(s, b))
    rhs = np.vdot(oracle.apply_H(s, a), b)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_constant_potential_shifts_spectrum(cfg1_system):
    s = cfg1_system
    rng = np.random.default_rng(4)
    c = _rand(rng, s.npw)
    shifted = oracle.System(L=s.L, N=s.N, miller=s.miller, vloc_r=s.vloc_r + 0.37,
                            beta=s.beta, dij=s.dij)
    d = oracle.apply_H(shifted, c) - oracle.apply_H(s, c)
    assert np.abs(d - 0.37 * c).max() < 1e-13


def test_spectrum_invariant_under_rigid_translation():
    """Moving every atom by the same vector multiplies V(G) and beta(G) by the same
    phase exp(-i G.t): H' = U H U^+, so the spectrum is unchanged.  A sign slip
    between the local and the nonlocal structure factors would break this."""
    cfg = workloads.get_config("cfg1")
    m = workloads.miller_sphere(cfg.M2)
    t = np.array([0.31, -1.17, 0.58])
    orig = workloads.crystal.atom_positions

    def shifted_positions(c):
        return orig(c) + t

    s0 = oracle.build_system("cfg1")
    try:
        workloads.crystal.atom_positions = shifted_positions
        s1 = oracle.System(L=cfg.L, N=cfg.N, miller=m, vloc_r=workloads.vloc_r(cfg),
                           beta=workloads.beta_projectors(cfg, m), dij=workloads.dij(cfg))
    finally:
        workloads.crystal.atom_positions = orig
    w0 = np.linalg.eigvalsh(oracle.dense_H(s0))
    w1 = np.linalg.eigvalsh(oracle.dense_H(s1))
    assert np.abs(w0 - w1).max() < 1e-12
    assert np.abs(s0.vloc_r - s1.vloc_r).max() > 1e-3   # the potential really moved


def test_local_potential_fourier_coefficients(cfg1_system):
    """The oracle's forward FFT of V_loc(r) returns the Gaussian form factor times the
    structure factor, (1/Omega) vhat(|G|) sum_a exp(-i G.R_a), inside the density sphere."""
    s = cfg1_system
    cfg = workloads.get_config("cfg1")
    VG = oracle.hamiltonian.potential_fourier(s, s.vloc_r)
    R = workloads.atom_positions(cfg)
    for m in ([0, 0, 0], [1, 1, 1], [2, 0, 0], [-3, 1, 2], [4, -4, 0]):
        G = s.G[0] * 0 + (2 * np.pi / s.L) * np.array(m, float)
        q2 = G @ G
        vhat = -cfg.V0 * (2 * np.pi * cfg.sigma ** 2) ** 1.5 * np.exp(-0.5 * q2 * cfg.sigma ** 2)
        expect = vhat * np.exp(-1j * (R @ G)).sum() / s.omega
        got = VG[tuple(np.mod(m, s.N))]
        assert abs(got - expect) < 1e-13


def test_projectors_normalised():
    """Each Gaussian KB projector is L2-normalised in real space; on the sphere its
    norm is 1 minus the (tiny) tail beyond the cutoff."""
    cfg = workloads.get_config("cfg2")
    m = workloads.miller_sphere(cfg.M2)
    beta = workloads.beta_projectors(cfg, m[:, :])
    n = (np.abs(beta) ** 2).sum(1)
    assert np.all(np.abs(n - 1.0) < 1e-3)
