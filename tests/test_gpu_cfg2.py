"""GPU parity at the 64-atom crystal's full size (72^3 grid, 22,575 plane waves,
128 bands, 256 KB projectors), in a 2048-slot context (full-width launches).

The oracle's valence states and its PCG responses of perturbations 0 and 1
over all 128 bands (Delta n, the chi0 block, four sampled Delta psi) are
stored in tests/oracle_data/ by tests/golden/make_valence_cache.py and
make_response_cache.py (oracle only); both sides use the same valence states.
"""
import numpy as np
import pytest

import oracle
import oracle_store
import workloads

pytestmark = pytest.mark.gpu

CFG = workloads.get_config("cfg2")


@pytest.fixture(scope="module")
def ref():
    eps, psi = oracle_store.valence("cfg2")
    s = oracle.build_system("cfg2")
    return s, eps, psi


@pytest.fixture(scope="module")
def resp():
    return oracle_store.load("cfg2", "response")


@pytest.fixture(scope="module")
def sth():
    import paper_2203_05623_amd as P
    ctx = P.sth_create(device=0, max_slots=2048)
    yield P, ctx
    P.sth_destroy(ctx)


@pytest.fixture(scope="module")
def sys2(sth, ref):
    P, ctx = sth
    s, eps, psi = ref
    nv = CFG.nv
    return P.sth_set_system(ctx, CFG.L, CFG.N, s.miller, s.vloc_r, s.beta, s.dij, psi[:nv],
                            eps[:nv])


@pytest.mark.parametrize("alg", ["lobpcg", "chfsi"])
def test_valence_matches_oracle(sth, ref, alg, monkeypatch):
    """Device eigensolver (block LOBPCG, or Chebyshev-filtered subspace
    iteration) vs the oracle's LOBPCG: eigenvalues are gauge invariant."""
    P, ctx = sth
    s, eps, psi = ref
    monkeypatch.setenv("STH_VALENCE", alg)
    e, v, res, its = P.sth_valence(ctx, CFG.L, CFG.N, s.miller, s.vloc_r, s.beta, s.dij,
                                   CFG.nv + 1, tol=1e-10)
    print(alg, "device valence: iterations", its, "residual", res)
    assert res <= 1e-10
    err = np.abs(e - eps[:CFG.nv + 1]).max()
    print("eigenvalue max abs diff", err, "gap", e[CFG.nv] - e[CFG.nv - 1])
    assert err < 1e-10


@pytest.fixture(scope="module")
def oracle_samples(resp):
    return {(int(j), int(v)): x for (j, v), x in zip(resp["samples"], resp["dpsi_samples"])}


@pytest.mark.parametrize("precision,tol,bound", [("fp64", 1e-12, 1e-10), ("mixed", 1e-8, 1e-6),
                                                 ("mixed-bf16", 1e-8, 1e-6)])
def test_sampled_solves_match_oracle(sth, ref, resp, sys2, oracle_samples, precision, tol,
                                    bound):
    P, ctx = sth
    s, eps, psi = ref
    npert = 2
    dv = workloads.dv_block(CFG, range(npert))
    prec = {"fp64": P.STH_FP64, "mixed": P.STH_MIXED, "mixed-bf16": P.STH_MIXED_BF16}[precision]
    t = P.sth_submit_solves(ctx, sys2, dv, np.arange(CFG.nv), tol=tol, precision=prec,
                            want_dpsi=True)
    assert P.sth_wait(ctx, t, 300.0)
    info = P.sth_poll(ctx, t)
    iters, resid, status, lat = P.sth_fetch_stats(ctx, t, npert * CFG.nv)
    print(precision, "iters mean/max", iters.mean(), iters.max(), "max resid", resid.max(),
          "op apps", info["op_applications"], "fp32", info["op_applications_fp32"])
    assert np.all(status == 0) and resid.max() <= tol
    dpsi = np.empty((npert, CFG.nv, s.npw), np.complex128)
    P.sth_fetch_dpsi(ctx, t, dpsi)
    for (j, v), x in oracle_samples.items():
        rel = np.linalg.norm(dpsi[j, v] - x) / np.linalg.norm(x)
        print(precision, "sample", (j, v), "rel err", rel)
        assert rel < bound
    # every solution is orthogonal to the valence manifold
    ov = np.abs(np.einsum("vg,jwg->jwv", psi[:CFG.nv].conj(), dpsi)).max()
    assert ov < 1e-10 * np.abs(dpsi).max() * np.sqrt(s.npw)
    # Delta n of both perturbations over all 128 bands and the chi0 block
    dn = np.empty((npert, CFG.N, CFG.N, CFG.N))
    P.sth_fetch_drho(ctx, t, dn)
    M, S, lam = P.sth_chi0_block(ctx, t, npert)
    P.sth_release_ticket(ctx, t)
    ref_dn = resp["drho"]
    e_dn = np.abs(dn - ref_dn).max() / np.abs(ref_dn).max()
    e_m = np.abs(M - resp["M"]).max() / np.abs(resp["M"]).max()
    e_l = np.abs(lam - resp["lam"]).max() / np.abs(resp["lam"]).max()
    print(precision, f"dn {e_dn:.2e}, M {e_m:.2e}, chi0 eigenvalues {e_l:.2e}")
    assert e_dn < bound and e_m < bound and e_l < bound
    assert np.allclose(S, resp["S"], rtol=1e-13, atol=0)
