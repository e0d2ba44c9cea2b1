"""Pins of the oracle's dense chi_bar0 = v^{1/2} chi0 v^{1/2} (CPU only).

What fixes the dense sum-over-states matrix independently of its own formula:
  * applied to a real, band-limited Delta V it gives the same Delta n as the
    Sternheimer route (dense LU solves of the projected equation for every
    valence band, then the density response), on a small basis where every
    conduction state is in the sum;
  * it is Hermitian and negative semidefinite (a sum of |<c|Delta V|v>|^2 terms
    over negative energy denominators);
  * the density sphere holds every sum of two wave-function sphere vectors.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import pdep


@pytest.fixture(scope="module")
def small():
    """Config-1 crystal on a small sphere (|m|^2 <= 6, 57 plane waves): all states dense."""
    s = oracle.build_system("cfg1", M2=6)
    H = oracle.dense_H(s)
    w, U = np.linalg.eigh(H)
    V = np.ascontiguousarray(U.T)
    nv = int(np.argmax(w[1:9] - w[:8])) + 1     # valence count at the widest low gap
    assert w[nv] - w[nv - 1] > 1e-3
    return s, H, w, V, nv


def _band_limited_real(s, mG, seed):
    rng = np.random.default_rng(seed)
    F = scipy.fft.fftn(rng.standard_normal((s.N,) * 3), norm="forward")
    keep = np.zeros(F.shape, bool)
    keep[tuple(np.mod(mG[:, k], s.N) for k in range(3))] = True
    F[~keep] = 0.0
    return np.real(scipy.fft.ifftn(F, norm="forward"))


def test_density_sphere_holds_products(small):
    s = small[0]
    mG = pdep.density_sphere(s)
    have = {tuple(m) for m in mG.tolist()} | {(0, 0, 0)}
    m = s.miller.astype(int)
    sums = (m[:, None, :] + m[None, :, :]).reshape(-1, 3)
    assert {tuple(x) for x in sums.tolist()} <= have
    assert len(have) == len(mG) + 1


def test_chi0_matrix_equals_sternheimer_response(small):
    s, H, w, V, nv = small
    mG = pdep.density_sphere(s)
    K = pdep.chi0_matrix(s, w, V, nv, mG)
    Psi, eps = V[:nv], w[:nv]
    for seed in (1, 2):
        dv = _band_limited_real(s, mG, seed)
        X = np.stack([oracle.solve_lu(H, Psi, eps[v], oracle.rhs(s, Psi, v, dv))
                      for v in range(nv)])
        dn_st = oracle.drho(s, Psi, X)
        dn_sos = pdep.apply_matrix_to_real(s, mG, K, dv)
        err = np.abs(dn_sos - dn_st).max() / np.abs(dn_st).max()
        print(f"nv {nv}, seed {seed}: sum over states vs Sternheimer {err:.2e}")
        assert err < 1e-11


def test_chibar0_hermitian_negative_semidefinite(small):
    s, H, w, V, nv = small
    _, K = pdep.chibar0_matrix(s, w, V, nv)
    assert np.abs(K - K.conj().T).max() < 1e-13 * np.abs(K).max()
    lam = np.linalg.eigvalsh(0.5 * (K + K.conj().T))
    assert lam.max() < 1e-12 * np.abs(lam).max()
    assert lam.min() < 0.0


# ---------------------------------------------------------------- Coulomb factor
def _gaussian_pair_hartree(L, q, sigma, d, mmax):
    """(Omega / 2) sum_{G != 0} v(G) |rho(G)|^2 with v(G) = coulomb_sqrt(G)^2, for
    rho = +q and -q normalised Gaussians of width sigma at +-d/2 along x in a cubic
    cell of edge L; rho(G) = (1 / Omega) int rho e^{-iG.r} dr."""
    from types import SimpleNamespace
    cell = SimpleNamespace(L=L)
    ax = np.arange(-mmax, mmax + 1)
    m = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    m = m[(m * m).sum(1) > 0]
    G = (2.0 * np.pi / L) * m.astype(np.float64)
    G2 = (G * G).sum(1)
    omega = L ** 3
    # e^{-iG.R1} - e^{-iG.R2} with R1,2 = +-d/2 x: -2i sin(G_x d / 2)
    rho2 = (q / omega) ** 2 * np.exp(-sigma ** 2 * G2) * 4.0 * np.sin(0.5 * G[:, 0] * d) ** 2
    v = pdep.coulomb_sqrt(cell, m) ** 2
    return 0.5 * omega * float((v * rho2).sum())


@pytest.mark.parametrize("L", [24.0, 36.0])
def test_coulomb_factor_gives_gaussian_pair_energy(L):
    """v^{1/2}(G)^2 must be the Fourier transform 4 pi / |G|^2 of 1/r: the periodic
    Hartree energy of a neutral pair of Gaussian charges then equals the
    closed-form energy of the isolated pair (two self-energies q^2 / (2 sigma
    sqrt(pi)) and the interaction -q^2 erf(d / (2 sigma)) / d) up to the
    interaction with the periodic images, which for a cubic lattice with the
    G = 0 term dropped is -2 pi p^2 / (3 Omega) at dipole order (p = q d).  A
    factor 4 pi / |G|, a missing Omega or a wrong reciprocal-lattice constant
    changes the energy by orders of magnitude."""
    from scipy.special import erf
    q, sigma, d = 1.0, 1.0, 3.0
    mmax = int(np.ceil(9.0 * L / (2.0 * np.pi * sigma)))     # e^{-sigma^2 G^2} < 1e-35 beyond
    e_per = _gaussian_pair_hartree(L, q, sigma, d, mmax)
    e_iso = q * q / (sigma * np.sqrt(np.pi)) - q * q * erf(d / (2.0 * sigma)) / d
    e_dip = -2.0 * np.pi * (q * d) ** 2 / (3.0 * L ** 3)
    print(f"L {L}: periodic {e_per:.10f}, isolated {e_iso:.10f}, dipole term {e_dip:.3e}, "
          f"rest {e_per - e_iso - e_dip:.3e}")
    assert abs(e_per - e_iso) < 2.0 * abs(e_dip)
    # beyond dipole order the image interaction falls off as d^4 / L^5
    assert abs(e_per - e_iso - e_dip) < 5.0 * q * q * d ** 4 / L ** 5


# ---------------------------------------------------------------- preconditioner
def test_tpa_preconditioner_limits(cfg1_system):
    """Teter-Payne-Allan diagonal (Phys. Rev. B 40, 12255): K = 1 at G = 0 with the
    first three derivatives in x = T / E_kin vanishing (1 - K ~ 16 x^4 / 27), 0 < K <= 1,
    and K ~ 1 / (2 x) at high kinetic energy (the inverse of (T - eps) / E_kin up to the
    factor 2 the polynomial is built with)."""
    s = cfg1_system
    T = oracle.kinetic(s)
    g = int(np.argmax(T))
    psi = np.zeros(s.npw, complex)
    psi[g] = 1.0                       # <psi|T|psi> = T(G_g) > the 0.1 Ha floor
    ek = T[g]
    K = oracle.tpa_precond(s, psi)
    x = T / ek
    assert np.all(K > 0.0) and np.all(K <= 1.0)
    g0 = int(np.argmin(T))
    assert T[g0] == 0.0 and K[g0] == 1.0
    small = (x > 0) & (x < 0.05)
    assert small.any()
    np.testing.assert_allclose((1.0 - K[small]) / x[small] ** 4, 16.0 / 27.0, rtol=0.2)
    # the asymptotic regime: a wide sphere (T up to ~75 Ha) and a band whose kinetic
    # energy sits at the 0.1 Ha floor
    import workloads
    wide = oracle.System(L=s.L, N=s.N, miller=workloads.miller_sphere(400),
                         vloc_r=np.zeros((s.N,) * 3), beta=np.zeros((0, 1), complex),
                         dij=np.zeros(0))
    Tw = oracle.kinetic(wide)
    psi0 = np.zeros(wide.npw, complex)
    psi0[int(np.argmin(Tw))] = 1.0
    K0 = oracle.tpa_precond(wide, psi0)
    x0 = Tw / 0.1
    big = x0 > 100.0
    assert big.any()
    np.testing.assert_allclose(2.0 * x0[big] * K0[big], 1.0, atol=1.5 / x0[big].min())
