"""GPU parity of the HIP path against the oracle on the tiny crystal (config 1).

Calls go through the C-ABI (ctypes binding).  Tolerances: FP64 throughout;
H.psi to 1e-12 relative (two FFT routes in FP64), Delta psi / Delta n / chi0 to
1e-10 relative at solve tolerance 1e-12 (the workload's FP64 parity bound).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

NV = 8


@pytest.fixture(scope="module")
def sth():
    import paper_2203_05623_amd as P
    ctx = P.sth_create(device=0, max_slots=256)
    yield P, ctx
    P.sth_destroy(ctx)


@pytest.fixture(scope="module")
def cfg1(cfg1_system, cfg1_dense):
    H, w, V = cfg1_dense
    cfg = workloads.get_config("cfg1")
    return cfg, cfg1_system, H, w[:NV], np.ascontiguousarray(V[:NV])


@pytest.fixture(scope="module")
def sys1(sth, cfg1):
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, Psi, eps)
    return sid


def test_apply_h_matches_oracle(sth, cfg1, sys1):
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    rng = np.random.default_rng(11)
    c = rng.standard_normal((37, s.npw)) + 1j * rng.standard_normal((37, s.npw))
    got = P.sth_apply_h(ctx, sys1, c)
    ref = oracle.apply_H(s, c)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("apply_h rel err", err)
    assert err < 1e-12


def test_solves_match_oracle(sth, cfg1, sys1):
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    npert = cfg.npert
    dv = workloads.dv_block(cfg, range(npert))
    bands = np.arange(NV)
    t = P.sth_submit_solves(ctx, sys1, dv, bands, tol=1e-12, want_dpsi=True)
    assert P.sth_wait(ctx, t, 120.0)
    info = P.sth_poll(ctx, t)
    assert info["n_converged"] == npert * NV
    dpsi = np.empty((npert, NV, s.npw), np.complex128)
    P.sth_fetch_dpsi(ctx, t, dpsi)
    drho = np.empty((npert, cfg.N, cfg.N, cfg.N))
    P.sth_fetch_drho(ctx, t, drho)
    iters, resid, status, lat = P.sth_fetch_stats(ctx, t, npert * NV)
    assert np.all(status == 0) and np.all(resid <= 1e-12)
    print("iters min/mean/max", iters.min(), iters.mean(), iters.max())
    # oracle: dense LU solve of the projected equation for every (j, v)
    X = np.empty_like(dpsi)
    for v in range(NV):
        B = np.stack([oracle.rhs(s, Psi, v, dv[j]) for j in range(npert)], 1)
        X[:, v] = oracle.solve_lu(H, Psi, eps[v], B).T
    rel = np.linalg.norm(dpsi - X, axis=2) / np.linalg.norm(X, axis=2)
    print("dpsi max rel err", rel.max())
    assert rel.max() < 1e-10
    dn_ref = np.stack([oracle.drho(s, Psi, X[j]) for j in range(npert)])
    err = np.abs(drho - dn_ref).max() / np.abs(dn_ref).max()
    print("drho rel err", err)
    assert err < 1e-10
    M, S, lam = P.sth_chi0_block(ctx, t, npert)
    lam_ref, M_ref, S_ref = oracle.chi0_block(s, dv, dn_ref)
    print("chi0 lam", lam[:4], lam_ref[:4])
    assert np.abs(M - M_ref).max() < 1e-10 * np.abs(M_ref).max()
    assert np.abs(S - S_ref).max() < 1e-12
    assert np.abs(lam - lam_ref).max() < 1e-10 * np.abs(lam_ref).max()
    P.sth_release_ticket(ctx, t)


@pytest.mark.parametrize("alg", ["lobpcg", "chfsi"])
def test_valence_lobpcg_matches_dense(sth, cfg1, cfg1_dense, alg, monkeypatch):
    """Device eigenpairs of H (block LOBPCG, or Chebyshev-filtered subspace
    iteration, forced through STH_VALENCE) vs dense diagonalisation (oracle)."""
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    H_, w, V = cfg1_dense
    monkeypatch.setenv("STH_VALENCE", alg)
    e, psi, res, its = P.sth_valence(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij,
                                     NV + 1, tol=1e-11)
    print(alg, "valence iters", its, "residual", res)
    assert res <= 1e-11
    assert np.abs(e - w[:NV + 1]).max() < 1e-11
    R = psi @ H.T - e[:, None] * psi
    assert np.linalg.norm(R, axis=1).max() < 1e-10
    assert np.abs(psi.conj() @ psi.T - np.eye(NV + 1)).max() < 1e-12


@pytest.mark.parametrize("form", ["mixed", "mixed-bf16"])
def test_mixed_precision_matches_oracle(sth, cfg1, sys1, form):
    """Mixed precision on the tiny crystal (FP32 FFT / H.psi inside CG with the
    projector GEMMs on FP32 MFMA, or on BF16 MFMA with hi/lo split operands; FP64
    residuals and defect correction): true residual 1e-8, Delta psi and chi0
    eigenvalues within 1e-6 of the FP64 oracle."""
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    npert = cfg.npert
    dv = workloads.dv_block(cfg, range(npert))
    prec = P.STH_MIXED if form == "mixed" else P.STH_MIXED_BF16
    t = P.sth_submit_solves(ctx, sys1, dv, np.arange(NV), tol=1e-8, precision=prec,
                            want_dpsi=True)
    assert P.sth_wait(ctx, t, 120.0)
    info = P.sth_poll(ctx, t)
    dpsi = np.empty((npert, NV, s.npw), np.complex128)
    P.sth_fetch_dpsi(ctx, t, dpsi)
    iters, resid, status, lat = P.sth_fetch_stats(ctx, t, npert * NV)
    print(form, ": iters mean", iters.mean(), "op apps", info["op_applications"],
          "fp32", info["op_applications_fp32"], "max resid", resid.max())
    assert np.all(status == 0) and resid.max() <= 1e-8
    assert info["op_applications_fp32"] > 0
    X = np.empty_like(dpsi)
    for v in range(NV):
        B = np.stack([oracle.rhs(s, Psi, v, dv[j]) for j in range(npert)], 1)
        X[:, v] = oracle.solve_lu(H, Psi, eps[v], B).T
    rel = np.linalg.norm(dpsi - X, axis=2) / np.linalg.norm(X, axis=2)
    print(form, "dpsi max rel err", rel.max())
    assert rel.max() < 1e-6
    dn_ref = np.stack([oracle.drho(s, Psi, X[j]) for j in range(npert)])
    M, S, lam = P.sth_chi0_block(ctx, t, npert)
    lam_ref, _, _ = oracle.chi0_block(s, dv, dn_ref)
    err = np.abs(lam - lam_ref).max() / np.abs(lam_ref).max()
    print(form, "chi0 eigenvalue rel err", err)
    assert err < 1e-6
    P.sth_release_ticket(ctx, t)


def test_solve_status_reports_maxit(sth, cfg1, sys1):
    """Failure handling forced from the host: maxit = 3 gives per-solve MAXIT status
    with the last iterate's residual, and the ticket still completes."""
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    dv = workloads.dv_block(cfg, range(2))
    t = P.sth_submit_solves(ctx, sys1, dv, np.arange(NV), tol=1e-12, maxit=3)
    assert P.sth_wait(ctx, t, 60.0)
    iters, resid, status, lat = P.sth_fetch_stats(ctx, t, 2 * NV)
    assert np.all(status == P._lib.SOLVE_MAXIT)
    assert np.all(iters == 3) and np.all(resid > 1e-12)
    P.sth_release_ticket(ctx, t)


@pytest.mark.parametrize("form", ["mixed", "mixed-bf16"])
def test_maxit_reports_true_fp64_residual(sth, cfg1, sys1, form):
    """A mixed-precision solve stopped by maxit inside the recurrence reports the
    true FP64 residual ||b - A x|| / ||b|| of the iterate it returns (recomputed
    here with the oracle's dense operator), not the recursive residual of the
    FP32 / BF16 inner operator."""
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    prec = {"mixed": P.STH_MIXED, "mixed-bf16": P.STH_MIXED_BF16}[form]
    dv = workloads.dv_block(cfg, range(2))
    t = P.sth_submit_solves(ctx, sys1, dv, np.arange(NV), tol=1e-12, maxit=4, precision=prec,
                            want_dpsi=True)
    assert P.sth_wait(ctx, t, 60.0)
    iters, resid, status, lat = P.sth_fetch_stats(ctx, t)
    assert np.all(status == P._lib.SOLVE_MAXIT)
    dpsi = np.empty((2, NV, s.npw), np.complex128)
    P.sth_fetch_dpsi(ctx, t, dpsi)
    n = s.npw
    Pc = np.eye(n) - Psi.T @ Psi.conj()
    for j in range(2):
        for v in range(NV):
            b = oracle.rhs(s, Psi, v, dv[j])
            A = Pc @ (H - eps[v] * np.eye(n)) @ Pc
            true = np.linalg.norm(b - A @ dpsi[j, v]) / np.linalg.norm(b)
            k = j * NV + v
            assert abs(resid[k] - true) <= 1e-6 * true, (j, v, resid[k], true)
    P.sth_release_ticket(ctx, t)


def test_invalid_arguments_are_errors(sth, cfg1, sys1):
    P, ctx = sth
    cfg, s, H, eps, Psi = cfg1
    dv = workloads.dv_block(cfg, range(1))
    with pytest.raises(P.SthError) as e:
        P.sth_submit_solves(ctx, sys1, dv, np.array([0, 0]))        # repeated band
    assert e.value.code == P._lib.STH_E_INVALID
    with pytest.raises(P.SthError) as e:
        P.sth_submit_solves(ctx, sys1 + 99, dv, np.arange(2))       # unknown system
    assert e.value.code == P._lib.STH_E_NOT_FOUND
    bad = s.miller.copy()
    bad[1] = bad[0]                                                  # duplicate Miller index
    with pytest.raises(P.SthError) as e:
        P.sth_set_system(ctx, cfg.L, cfg.N, bad, s.vloc_r, s.beta, s.dij, Psi, eps)
    assert e.value.code == P._lib.STH_E_INVALID
    t = P.sth_submit_solves(ctx, sys1, dv, np.arange(2), tol=1e-10)
    assert P.sth_wait(ctx, t, 60.0)
    P.sth_release_ticket(ctx, t)
    with pytest.raises(P.SthError) as e:
        P.sth_poll(ctx, t)
    assert e.value.code == P._lib.STH_E_NOT_FOUND


def test_graph_replay_matches_direct_launches(cfg1, tmp_path, monkeypatch):
    """With fewer slots than solves the server reaches the steady state where the
    captured hipGraph of CG iterations is replayed (with the server's own eager
    refills, retirements and synchronisations between replays).  The result must
    equal, bit for bit, a run with direct launches (deterministic reductions).
    Both runs share one autotuner cache, so that they use the same FFT plans and
    GEMM split (a timing-based choice could differ between two contexts)."""
    import paper_2203_05623_amd as P
    cfg, s, H, eps, Psi = cfg1
    dv = workloads.dv_block(cfg, range(cfg.npert))
    out = {}
    monkeypatch.setenv("STH_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    for mode in ("1", "0"):
        monkeypatch.setenv("STH_GRAPHS", mode)
        ctx = P.sth_create(device=0, max_slots=64)
        try:
            sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, Psi, eps)
            for prec in (P.STH_FP64, P.STH_MIXED, P.STH_MIXED_BF16):
                t = P.sth_submit_solves(ctx, sid, dv, np.arange(NV), tol=1e-10, precision=prec,
                                        want_dpsi=True)
                assert P.sth_wait(ctx, t, 120.0)
                info = P.sth_poll(ctx, t)
                x = np.empty((cfg.npert, NV, s.npw), np.complex128)
                P.sth_fetch_dpsi(ctx, t, x)
                out[(mode, prec)] = (x, info["graph_replays"])
                P.sth_release_ticket(ctx, t)
        finally:
            P.sth_destroy(ctx)
    for prec in (P.STH_FP64, P.STH_MIXED, P.STH_MIXED_BF16):
        xg, ng = out[("1", prec)]
        xd, nd = out[("0", prec)]
        print("precision", prec, "graph replays", ng, "direct", nd)
        assert ng > 0 and nd == 0
        assert np.array_equal(xg, xd)
