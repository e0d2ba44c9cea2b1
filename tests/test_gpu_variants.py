"""GPU parity of every FFT-stage variant the autotuner can pick.

The autotuner keeps the fastest (radix plan, plane kernel form, z-stick kernel
form) per precision, so a normal run exercises only one of them.  Here every radix
plan and every kernel form of both stages (plane: workgroup, wave, strip,
persistent and compact-row forms; z-sticks: workgroup and wave forms) is forced
through the tuning cache (STH_TUNE_CACHE) in FP64 and in FP32 and checked
against the oracle: H.psi in FP64 (1e-12 relative) and mixed-precision solves,
whose inner operator uses the FP32 variant (1e-6 relative on Delta psi at true
residual 1e-8).  On config 1 also FP64
solves at 1e-12 with their Delta n (1e-10), which run psi_v(r) and Delta n
through the FP64 form.  Config 1 (24^3, plans (8, 3) and (4, 6)) and the
benchmark system (72^3, plans (8, 9) and (9, 8)).
"""
import numpy as np
import pytest

import oracle
import oracle_store
import tune_force
import workloads

pytestmark = pytest.mark.gpu

VARIANTS = [(plan, kind) for plan in (0, 1) for kind in (0, 1, 2, 3, 4)]


def _systems(P, ctx, monkeypatch, tmp_path, cfg, s, psi, eps, nv):
    """Yields (plan, kind, system id) with the variant forced (z-stick forms
    alternate with the plane form, FP64 and FP32 opposite)."""
    info = tune_force.shape_info(P, ctx, cfg, s, psi, eps)
    for plan, kind in VARIANTS:
        path = tmp_path / f"tune_{plan}_{kind}.jsonl"
        sid = tune_force.system_with(P, ctx, monkeypatch, path, cfg, s, psi, eps,
                                     ((plan, kind, kind % 2), (plan, kind, 1 - kind % 2)), info)
        yield plan, kind, sid
        P.sth_release_system(ctx, sid)


def test_variants_cfg1(cfg1_system, cfg1_dense, monkeypatch, tmp_path):
    import paper_2203_05623_amd as P
    cfg = workloads.get_config("cfg1")
    s = cfg1_system
    H, w, V = cfg1_dense
    nv = cfg.nv
    eps, psi = w[:nv], np.ascontiguousarray(V[:nv])
    rng = np.random.default_rng(21)
    c = rng.standard_normal((19, s.npw)) + 1j * rng.standard_normal((19, s.npw))
    ref_h = oracle.apply_H(s, c)
    dv = workloads.dv_block(cfg, range(2))
    ref_x = np.array([[oracle.solve_lu(H, psi, eps[v], oracle.rhs(s, psi, v, dv[j]))
                       for v in range(nv)] for j in range(2)])
    ref_dn = np.stack([oracle.drho(s, psi, ref_x[j]) for j in range(2)])
    ctx = P.sth_create(device=0, max_slots=64)
    try:
        for plan, kind, sid in _systems(P, ctx, monkeypatch, tmp_path, cfg, s, psi, eps, nv):
            got = P.sth_apply_h(ctx, sid, c)
            e_h = np.abs(got - ref_h).max() / np.abs(ref_h).max()
            t = P.sth_submit_solves(ctx, sid, dv, np.arange(nv), tol=1e-8,
                                    precision=P.STH_MIXED, want_dpsi=True)
            assert P.sth_wait(ctx, t, 120.0)
            x = np.empty((2, nv, s.npw), np.complex128)
            P.sth_fetch_dpsi(ctx, t, x)
            P.sth_release_ticket(ctx, t)
            e_x = max(np.linalg.norm(x[j, v] - ref_x[j, v]) / np.linalg.norm(ref_x[j, v])
                      for j in range(2) for v in range(nv))
            t = P.sth_submit_solves(ctx, sid, dv, np.arange(nv), tol=1e-12, want_dpsi=True)
            assert P.sth_wait(ctx, t, 120.0)
            P.sth_fetch_dpsi(ctx, t, x)
            dn = np.empty((2, cfg.N, cfg.N, cfg.N))
            P.sth_fetch_drho(ctx, t, dn)
            P.sth_release_ticket(ctx, t)
            e_x64 = max(np.linalg.norm(x[j, v] - ref_x[j, v]) / np.linalg.norm(ref_x[j, v])
                        for j in range(2) for v in range(nv))
            e_dn = np.abs(dn - ref_dn).max() / np.abs(ref_dn).max()
            print(f"cfg1 plan {plan} kind {kind}: H.psi {e_h:.2e}, mixed dpsi {e_x:.2e}, "
                  f"FP64 dpsi {e_x64:.2e}, dn {e_dn:.2e}")
            assert e_h < 1e-12
            assert e_x < 1e-6
            assert e_x64 < 1e-10 and e_dn < 1e-10
    finally:
        P.sth_destroy(ctx)


def test_variants_cfg2(monkeypatch, tmp_path):
    import paper_2203_05623_amd as P
    cfg = workloads.get_config("cfg2")
    s = oracle.build_system("cfg2")
    nv = cfg.nv
    eps, psi = oracle_store.valence("cfg2")
    eps, psi = eps[:nv], psi[:nv]
    rng = np.random.default_rng(22)
    c = rng.standard_normal((5, s.npw)) + 1j * rng.standard_normal((5, s.npw))
    ref_h = oracle.apply_H(s, c)
    j, v = 0, 127
    dvj = workloads.dv_r(cfg, j)
    ref_x, _, _, st = oracle.pcg_solve(s, psi, eps, v, oracle.rhs(s, psi, v, dvj), tol=1e-12)
    assert st == 0
    ctx = P.sth_create(device=0, max_slots=256)
    try:
        for plan, kind, sid in _systems(P, ctx, monkeypatch, tmp_path, cfg, s, psi, eps, nv):
            got = P.sth_apply_h(ctx, sid, c)
            e_h = np.abs(got - ref_h).max() / np.abs(ref_h).max()
            t = P.sth_submit_solves(ctx, sid, dvj[None], np.array([v]), tol=1e-8,
                                    precision=P.STH_MIXED, want_dpsi=True)
            assert P.sth_wait(ctx, t, 120.0)
            x = np.empty((1, 1, s.npw), np.complex128)
            P.sth_fetch_dpsi(ctx, t, x)
            P.sth_release_ticket(ctx, t)
            e_x = np.linalg.norm(x[0, 0] - ref_x) / np.linalg.norm(ref_x)
            print(f"cfg2 plan {plan} kind {kind}: H.psi {e_h:.2e}, mixed dpsi {e_x:.2e}")
            assert e_h < 1e-12
            assert e_x < 1e-6
    finally:
        P.sth_destroy(ctx)
