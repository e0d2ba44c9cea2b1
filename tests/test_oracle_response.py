"""Pins of the oracle's Sternheimer solve, density response and chi0 block (CPU only).

What fixes each result independently of the oracle's own formulas:
  * the sum over every conduction state (first-order perturbation theory) and
    a dense LU solve of the projected equation are two different routes to the
    same Delta psi;
  * for free electrons the solution has a closed form in the Fourier
    coefficients of Delta V;
  * Delta n is the derivative of the ground-state density of H + lambda dV with
    respect to lambda (finite differences of exact diagonalisations), and
    M_jj = <dV_j|chi0|dV_j> is the second derivative of the band energy;
  * charge neutrality, linearity, gauge invariance inside a degenerate shell,
    reciprocity (M symmetric) and negative semidefiniteness of chi0.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads
from oracle.hamiltonian import dense_potential_matrix, kinetic
from oracle.response import project_c


NV = 8


@pytest.fixture(scope="module")
def cfg1_setup(cfg1_system, cfg1_dense):
    H, w, V = cfg1_dense
    cfg = workloads.get_config("cfg1")
    dv = workloads.dv_block(cfg, range(4))
    return cfg1_system, H, w, V, dv


@pytest.fixture(scope="module")
def cfg1_dpsi(cfg1_setup):
    """Delta psi_jv [4, NV, npw] of config 1 by dense LU solves."""
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    X = np.empty((len(dv), NV, s.npw), complex)
    for v in range(NV):
        B = np.stack([oracle.rhs(s, Psi, v, dv[j]) for j in range(len(dv))], 1)
        X[:, v] = oracle.solve_lu(H, Psi, eps[v], B).T
    return X


def test_sum_over_states_equals_lu(cfg1_setup):
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    for j in range(2):
        for v in (0, 3, 7):
            b = oracle.rhs(s, Psi, v, dv[j])
            x_lu = oracle.solve_lu(H, Psi, eps[v], b)
            u = oracle.hamiltonian.apply_local(s, dv[j], Psi[v])
            x_sos = oracle.solve_sum_over_states(w, V, NV, v, u)
            assert np.linalg.norm(x_lu - x_sos) / np.linalg.norm(x_sos) < 1e-12
            # orthogonal to the valence manifold
            assert np.abs(Psi.conj() @ x_lu).max() < 1e-12 * np.linalg.norm(x_lu)


def test_pcg_matches_dense_solve(cfg1_setup):
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    for j, v in ((0, 0), (1, 5), (3, 7)):
        b = oracle.rhs(s, Psi, v, dv[j])
        x_lu = oracle.solve_lu(H, Psi, eps[v], b)
        x, it, rel, status = oracle.pcg_solve(s, Psi, eps, v, b, tol=1e-12)
        assert status == 0 and rel <= 1e-12
        assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-10
        assert 5 < it < 200


def test_pcg_reports_max_iterations(cfg1_setup):
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    b = oracle.rhs(s, Psi, 2, dv[0])
    x, it, rel, status = oracle.pcg_solve(s, Psi, eps, 2, b, tol=1e-12, maxit=3)
    assert status == 1 and it == 3 and rel > 1e-12


def test_free_electron_closed_form():
    """V = 0, no projectors, valence = the closed shell |m|^2 <= 1 (7 plane waves):
    Delta psi_v(G) = -dV(G - G_v) / (|G|^2/2 - |G_v|^2/2) for G outside the shell.
    The oracle's closed form is checked against the expression written out here,
    against the dense LU solve of the projected equation and against its PCG;
    a constant potential c shifts H and eps_v alike and leaves it unchanged."""
    s = oracle.build_free_electron_system("cfg1")
    cfg = workloads.get_config("cfg1")
    m = s.miller.astype(int)
    msq = (m * m).sum(1)
    val = np.flatnonzero(msq <= 1)
    assert len(val) == 7
    Psi = np.zeros((7, s.npw), complex)
    Psi[np.arange(7), val] = 1.0
    T = kinetic(s)
    dv = workloads.dv_r(cfg, 3)
    dVG = np.fft.fftn(dv) / s.N ** 3
    for c in (0.0, -0.3):
        sc = dataclasses.replace(s, vloc_r=np.full_like(s.vloc_r, c))
        eps = T[val] + c
        H = oracle.dense_H(sc)
        for v in range(7):
            d = np.mod(m - m[val[v]], s.N)
            expect = -dVG[d[:, 0], d[:, 1], d[:, 2]] / (T - T[val[v]] + (msq <= 1))
            expect[msq <= 1] = 0.0
            got = oracle.free_electron_response(sc, val, v, dv)
            assert np.abs(got - expect).max() < 1e-15 * np.abs(expect).max()
            b = oracle.rhs(sc, Psi, v, dv)
            x = oracle.solve_lu(H, Psi, eps[v], b)
            assert np.abs(x - got).max() < 1e-13 * max(1.0, np.abs(got).max())
            xp, _, rel, st = oracle.pcg_solve(sc, Psi, eps, v, b, tol=1e-12)
            assert st == 0 and np.linalg.norm(xp - got) < 1e-10 * np.linalg.norm(got)
    with pytest.raises(ValueError):   # |m|^2 <= 1 without one of its plane waves
        oracle.free_electron_response(s, val[:-1], 0, dv)


def _density_of(s, H):
    w, V = np.linalg.eigh(H)
    return oracle.density(s, np.ascontiguousarray(V[:, :NV].T)), w[:NV]


def test_drho_is_derivative_of_density(cfg1_setup, cfg1_dpsi):
    """Delta n_j = d n / d lambda of H + lambda dV_j, by central differences with
    Richardson extrapolation (error O(h^4)) over exact diagonalisations."""
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    j = 1
    dV = dense_potential_matrix(s, dv[j])
    dn = oracle.drho(s, Psi, cfg1_dpsi[j])

    def D(h):
        return (_density_of(s, H + h * dV)[0] - _density_of(s, H - h * dV)[0]) / (2 * h)

    h = 2e-3
    fd = (4 * D(h / 2) - D(h)) / 3
    assert np.abs(fd - dn).max() / np.abs(dn).max() < 1e-7
    # charge neutrality: the integral of Delta n vanishes
    assert abs(dn.sum() * s.omega / s.N ** 3) < 1e-12 * np.abs(dn).max() * s.omega


def test_chi0_block_second_derivative_and_symmetry(cfg1_setup, cfg1_dpsi):
    """M_ij = (Omega/N^3) sum_r dV_i Dn_j equals d^2 E_band / d lambda_i d lambda_j
    with E_band = f_s sum_v eps_v(H + sum lambda dV); M is symmetric and chi0 <= 0."""
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]
    nj = len(dv)
    dn = np.stack([oracle.drho(s, Psi, cfg1_dpsi[j]) for j in range(nj)])
    lam, M, S = oracle.chi0_block(s, dv, dn)
    assert np.abs(M - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.all(lam < 0)
    assert np.allclose(np.diag(S), 1.0, atol=1e-12)        # unit-norm perturbations

    dV = [dense_potential_matrix(s, dv[j]) for j in range(nj)]

    def E(Hm):
        return s.spin_factor * np.linalg.eigvalsh(Hm)[:NV].sum()

    h = 1e-2
    for i, j in ((0, 0), (2, 2), (0, 3)):
        if i == j:
            d2 = (E(H + h * dV[i]) - 2 * E(H) + E(H - h * dV[i])) / h ** 2
            d2h = (E(H + 0.5 * h * dV[i]) - 2 * E(H) + E(H - 0.5 * h * dV[i])) / (0.25 * h * h)
        else:
            def f(a, b, hh):
                return E(H + a * hh * dV[i] + b * hh * dV[j])
            d2 = (f(1, 1, h) - f(1, -1, h) - f(-1, 1, h) + f(-1, -1, h)) / (4 * h * h)
            hh = 0.5 * h
            d2h = (f(1, 1, hh) - f(1, -1, hh) - f(-1, 1, hh) + f(-1, -1, hh)) / (4 * hh * hh)
        rich = (4 * d2h - d2) / 3
        assert abs(rich - M[i, j]) < 1e-6 * abs(M[i, i])


def test_drho_linear_and_gauge_invariant(cfg1_setup):
    s, H, w, V, dv = cfg1_setup
    Psi, eps = V[:NV], w[:NV]

    def dn_of(P, e, pot):
        X = np.stack([oracle.solve_sum_over_states(w, np.vstack([P, V[NV:]]), NV, v,
                                                   oracle.hamiltonian.apply_local(s, pot, P[v]))
                      for v in range(NV)])
        return oracle.drho(s, P, X)

    a = dn_of(Psi, eps, dv[0])
    b = dn_of(Psi, eps, dv[1])
    c = dn_of(Psi, eps, dv[0] + 2.0 * dv[1])
    assert np.abs(c - (a + 2 * b)).max() < 1e-12 * np.abs(c).max()
    # bands 1..6 form a 6-fold degenerate shell: rotate them by a random unitary
    assert np.ptp(eps[1:7]) < 1e-10
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6)))
    P2 = Psi.copy()
    P2[1:7] = Q.T @ Psi[1:7]
    a2 = dn_of(P2, eps, dv[0])
    assert np.abs(a2 - a).max() < 1e-11 * np.abs(a).max()


def test_project_c_is_projector(cfg1_setup):
    s, H, w, V, dv = cfg1_setup
    Psi = V[:NV]
    rng = np.random.default_rng(6)
    y = rng.standard_normal(s.npw) + 1j * rng.standard_normal(s.npw)
    p1 = project_c(Psi, y)
    assert np.abs(project_c(Psi, p1) - p1).max() < 1e-14
    assert np.abs(Psi.conj() @ p1).max() < 1e-14
