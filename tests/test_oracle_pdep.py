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
