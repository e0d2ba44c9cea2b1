"""GPU parity of the batched Lanczos chains (sth_lanczos) against the oracle.

Chains of one orbital for a few real band-limited grid functions (stand-ins for
PDEP vectors), through the C-ABI, against oracle/lanczos.py on the same inputs:
alpha, beta and the tridiagonal eigenvalues within 1e-10 relative, the braket
<u_n|q^l_m> within 1e-10 of its largest entry, and the tridiagonal eigenvectors
up to the sign of each.  Config 1 (30 steps, 3 chains) and the benchmark system
(20 steps, 2 chains; oracle valence states from tests/oracle_data).
"""
import os

import numpy as np
import pytest
import scipy.fft

import oracle
import oracle_store
import workloads
from oracle import lanczos, pdep

pytestmark = pytest.mark.gpu
ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def _band_limited_real(s, seed):
    mG = pdep.density_sphere(s)
    rng = np.random.default_rng(seed)
    F = scipy.fft.fftn(rng.standard_normal((s.N,) * 3), norm="forward")
    keep = np.zeros(F.shape, bool)
    keep[tuple(np.mod(mG[:, k], s.N) for k in range(3))] = True
    F[~keep] = 0.0
    return np.real(scipy.fft.ifftn(F, norm="forward"))


def _compare(got, ref, tag):
    a, b, d, U, br = got
    ra, rb, rd, rU, rbr = ref
    e_a = np.abs(a - ra).max() / np.abs(ra).max()
    e_b = np.abs(b - rb).max() / np.abs(rb).max()
    e_d = np.abs(d - rd).max() / np.abs(rd).max()
    e_br = np.abs(br - rbr).max() / np.abs(rbr).max()
    sgn = np.sign(np.einsum("mlj,mlj->mj", U, rU))
    e_U = np.abs(U * sgn[:, None, :] - rU).max()
    print(f"{tag}: alpha {e_a:.2e} beta {e_b:.2e} d {e_d:.2e} braket {e_br:.2e} U {e_U:.2e}")
    assert e_a < 1e-10 and e_b < 1e-10 and e_d < 1e-10 and e_br < 1e-10
    assert e_U < 1e-7


def test_lanczos_cfg1(cfg1_system, cfg1_dense):
    import paper_2203_05623_amd as P
    cfg = workloads.get_config("cfg1")
    s = cfg1_system
    H, w, V = cfg1_dense
    phi = np.stack([_band_limited_real(s, 20 + k) for k in range(3)])
    ref = lanczos.lanczos_block(s, V[3], phi, 30)
    ctx = P.sth_create(device=0, max_slots=64)
    try:
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij,
                               np.ascontiguousarray(V[:cfg.nv]), w[:cfg.nv])
        got = P.sth_lanczos(ctx, sid, 3, phi, 30)
        _compare(got, ref, "cfg1")
    finally:
        P.sth_destroy(ctx)


def test_lanczos_cfg2():
    import paper_2203_05623_amd as P
    cfg = workloads.get_config("cfg2")
    eps, psi = oracle_store.valence("cfg2")
    s = oracle.build_system("cfg2")
    psi, eps = psi[:cfg.nv], eps[:cfg.nv]
    phi = np.stack([_band_limited_real(s, 30 + k) for k in range(2)])
    ref = lanczos.lanczos_block(s, psi[127], phi, 20)
    ctx = P.sth_create(device=0, max_slots=64)
    try:
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij,
                               np.ascontiguousarray(psi), eps)
        got = P.sth_lanczos(ctx, sid, 127, phi, 20)
        _compare(got, ref, "cfg2")
    finally:
        P.sth_destroy(ctx)
