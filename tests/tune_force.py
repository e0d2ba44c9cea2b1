"""Forces an FFT-stage variant on a system through the autotuner's cache file
(STH_TUNE_CACHE, JSON lines keyed by the system's shape), so that a test can
run a kernel form the autotuner would not pick."""


def write_choice(path, info, N, M, plan64, kind64, zkind64, plan32, kind32, zkind32):
    """Appends one cache entry for the system described by `info`
    (sth_system_info_get of the same system built without the cache)."""
    key = (f"gfx950 N={N} npw={info['npw']} nst={info['nsticks']} M={M} "
           f"slots={info['nslots']}")
    with open(path, "a") as f:
        f.write(f'{{"key": "{key}", "plan64": {plan64}, "kind64": {kind64}, '
                f'"zkind64": {zkind64}, "plan32": {plan32}, "kind32": {kind32}, '
                f'"zkind32": {zkind32}, "kchunk": {info["gemm_kchunk"]}}}\n')


def shape_info(P, ctx, cfg, s, psi, eps):
    """sth_system_info_get of the system built once without a cache file."""
    base = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, psi, eps)
    info = P.sth_system_info_get(ctx, base)
    P.sth_release_system(ctx, base)
    return info


def system_with(P, ctx, monkeypatch, path, cfg, s, psi, eps, choice, info=None):
    """Builds the system with `choice` = ((plan, kind, zkind) FP64, (...) FP32)
    forced through a cache file at `path`; returns the system id."""
    if info is None:
        info = shape_info(P, ctx, cfg, s, psi, eps)
    M = psi.shape[0] + s.beta.shape[0]
    (p64, k64, z64), (p32, k32, z32) = choice
    write_choice(path, info, cfg.N, M, p64, k64, z64, p32, k32, z32)
    monkeypatch.setenv("STH_TUNE_CACHE", str(path))
    sid = P.sth_set_system(ctx, cfg.L, cfg.N, s.miller, s.vloc_r, s.beta, s.dij, psi, eps)
    got = P.sth_system_info_get(ctx, sid)
    assert got["tuned_from_cache"] == 1
    assert (got["fft_plan_fp64"], got["plane_kernel_fp64"], got["zfft_kernel_fp64"]) == (p64, k64, z64)
    assert (got["fft_plan_fp32"], got["plane_kernel_fp32"], got["zfft_kernel_fp32"]) == (p32, k32, z32)
    monkeypatch.delenv("STH_TUNE_CACHE")
    return sid
