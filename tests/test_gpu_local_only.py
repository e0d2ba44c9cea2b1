"""GPU parity of a system without Kleinman-Bylander projectors (local potential only).

The config-1 crystal with its projectors removed (nproj = 0): the operator's KB
GEMMs have no rows, so each CG step is the FFT route plus the P_c projection.
Valence states from dense diagonalisation (oracle); 8 bands sit below a
0.28 Ha gap.  FP64 solves at 1e-12 against dense LU solves of the projected
equation (Delta psi and Delta n within 1e-10), and both mixed forms at 1e-8
(Delta psi within 1e-6), through the C-ABI.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
NV = 8


@pytest.fixture(scope="module")
def local_system(cfg1_system):
    s = cfg1_system
    s0 = dataclasses.replace(s, beta=np.zeros((0, s.npw), np.complex128), dij=np.zeros(0))
    H = oracle.dense_H(s0)
    w, U = np.linalg.eigh(H)
    assert w[NV] - w[NV - 1] > 0.1
    return s0, H, w[:NV], np.ascontiguousarray(U.T[:NV])


def test_local_only_solves(local_system):
    import paper_2203_05623_amd as P
    cfg = workloads.get_config("cfg1")
    s, H, eps, Psi = local_system
    dv = workloads.dv_block(cfg, range(4))
    ref = np.empty((len(dv), NV, s.npw), np.complex128)
    for v in range(NV):
        B = np.stack([oracle.rhs(s, Psi, v, dv[j]) for j in range(len(dv))], 1)
        ref[:, v] = oracle.solve_lu(H, Psi, eps[v], B).T
    ref_dn = np.stack([oracle.drho(s, Psi, ref[j]) for j in range(len(dv))])
    ctx = P.sth_create(device=0, max_slots=64)
    try:
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, Psi, eps)
        for prec, tol, bound in [(P.STH_FP64, 1e-12, 1e-10), (P.STH_MIXED, 1e-8, 1e-6),
                                 (P.STH_MIXED_BF16, 1e-8, 1e-6)]:
            t = P.sth_submit_solves(ctx, sid, dv, np.arange(NV), tol=tol, precision=prec,
                                    want_dpsi=True)
            assert P.sth_wait(ctx, t, 120.0)
            x = np.empty_like(ref)
            P.sth_fetch_dpsi(ctx, t, x)
            iters, resid, status, _ = P.sth_fetch_stats(ctx, t, len(dv) * NV)
            assert np.all(status == 0) and resid.max() <= tol
            err = max(np.linalg.norm(x[j, v] - ref[j, v]) / np.linalg.norm(ref[j, v])
                      for j in range(len(dv)) for v in range(NV))
            print(f"precision {prec}: iterations mean {iters.mean():.1f}, dpsi rel err {err:.2e}")
            assert err < bound
            if prec == P.STH_FP64:
                dn = np.empty((len(dv), cfg.N, cfg.N, cfg.N))
                P.sth_fetch_drho(ctx, t, dn)
                e_dn = np.abs(dn - ref_dn).max() / np.abs(ref_dn).max()
                print(f"dn rel err {e_dn:.2e}")
                assert e_dn < 1e-10
            P.sth_release_ticket(ctx, t)
    finally:
        P.sth_destroy(ctx)
