"""Pins of the oracle's Lanczos chains (CPU only).

What fixes the chains independently of the recurrence that builds them:
  * the chain vectors are orthonormal and Q H Q^H is the tridiagonal matrix of
    the alpha and beta (checked with the dense H of the tiny crystal);
  * the chain spans the Krylov space of H and the start vector: each H^k u
    (k < L) lies in span(Q);
  * the Lanczos form of the resolvent, ||u||^2 sum_l U_{1l}^2 / (d_l - z),
    approaches the dense <u|(H - z)^{-1}|u> as the chain grows (z off the real
    axis), the use the paper makes of it;
  * the braket of a chain with its own start vector is ||u|| on the first
    vector and zero on the others.
"""
import numpy as np
import pytest
import scipy.fft

import oracle
from oracle import lanczos, pdep

L = 30


def _band_limited_real(s, seed):
    mG = pdep.density_sphere(s)
    rng = np.random.default_rng(seed)
    F = scipy.fft.fftn(rng.standard_normal((s.N,) * 3), norm="forward")
    keep = np.zeros(F.shape, bool)
    keep[tuple(np.mod(mG[:, k], s.N) for k in range(3))] = True
    F[~keep] = 0.0
    return np.real(scipy.fft.ifftn(F, norm="forward"))


@pytest.fixture(scope="module")
def chains(cfg1_system, cfg1_dense):
    s = cfg1_system
    H, w, V = cfg1_dense
    phi = np.stack([_band_limited_real(s, 7), _band_limited_real(s, 8)])
    u = lanczos.start_vectors(s, V[3], phi)
    out = [lanczos.lanczos_chain(s, u[m], L) for m in range(2)]
    return s, H, u, phi, out


def test_chain_orthonormal_and_tridiagonalises_H(chains):
    s, H, u, phi, out = chains
    for a, b, Q in out:
        assert np.abs(Q.conj() @ Q.T - np.eye(L)).max() < 1e-12
        T = Q.conj() @ H @ Q.T
        Tl = lanczos.tridiagonal(a, b)
        assert np.abs(T - Tl).max() < 1e-11 * np.abs(Tl).max()


def test_chain_spans_krylov_space(chains):
    s, H, u, phi, out = chains
    a, b, Q = out[0]
    x = u[0] / np.linalg.norm(u[0])
    for k in range(12):
        resid = x - Q.T @ (Q.conj() @ x)
        assert np.linalg.norm(resid) < 1e-10, k
        x = H @ x
        x /= np.linalg.norm(x)


def test_resolvent_converges_to_dense(chains):
    s, H, u, phi, out = chains
    z = -0.2 + 1.0j
    exact = np.vdot(u[1], np.linalg.solve(H - z * np.eye(len(H)), u[1]))
    errs = []
    for nl in (10, 20, 30):
        a, b, Q = lanczos.lanczos_chain(s, u[1], nl)
        d, U = np.linalg.eigh(lanczos.tridiagonal(a, b))
        approx = b[0] ** 2 * np.sum(U[0] ** 2 / (d - z))
        errs.append(abs(approx - exact) / abs(exact))
    print("resolvent errors", errs)
    assert errs[2] < errs[0] and errs[2] < 1e-8


def test_block_braket_with_own_start(cfg1_system, cfg1_dense):
    s = cfg1_system
    H, w, V = cfg1_dense
    phi = np.stack([_band_limited_real(s, 9), _band_limited_real(s, 10)])
    A, B, D, U, braket = lanczos.lanczos_block(s, V[0], phi, 8)
    for m in range(2):
        assert abs(braket[m, m, 0] - B[m, 0]) < 1e-12 * B[m, 0]
        assert np.abs(braket[m, m, 1:]).max() < 1e-12 * B[m, 0]
        assert np.allclose(np.sort(D[m]), D[m])
