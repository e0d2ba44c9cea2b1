"""Throughput benchmark of the batched Sternheimer path on one MI355X.

A step is one pass of the whole hot path over one request: the right-hand
sides -P_c dV_j psi_v, the batched PCG solves of every (perturbation, band)
pair to a true relative residual of 1e-8, the density responses dn_j and the
chi0 block Rayleigh-Ritz.  Workload (default): the 64-atom synthetic supercell
on a 72^3 grid (22,575 plane waves, 128 valence bands from the device LOBPCG,
4 KB projectors per atom), 256 perturbations = 32,768 solves per step.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]

Prints one JSON line.  The CPU baseline is the oracle (plain FP64 NumPy PCG)
timed on a bounded sample of the same solves, run before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

METRIC = "Sternheimer solves/s, FP64 vs mixed at 1e-8 residual; p50/p99 solve latency"
MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6     # FP64 vector ALU and FP64 dense MFMA
MI355X_FP32_TFLOPS = 157.3    # FP32 vector ALU and FP32 dense MFMA
MI355X_BF16_TFLOPS = 2500.0   # BF16 dense MFMA
# (phase, precision) -> measured HBM bytes / algorithmic bytes of its kernel
# (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, see profiles/); entries are dropped
# whenever the kernel changes
HBM_OVER_ALGORITHMIC = {("plane", "fp64"): 1.0045,
                        # both mixed forms run the same plane kernels
                        ("plane", "mixed"): 1.0088, ("plane", "mixed-bf16"): 1.0088}
# --precision: FP64 solves; mixed (FP32 inner operator, FP32-MFMA projector
# GEMMs); mixed-bf16 (FP32 inner operator, BF16-MFMA hi/lo projector GEMMs)
PRECISIONS = {"fp64": lambda P: P.STH_FP64, "mixed": lambda P: P.STH_MIXED,
              "mixed-bf16": lambda P: P.STH_MIXED_BF16}


# ---------------------------------------------------------------- CPU baseline (oracle)
def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    name, cache, pairs, tol = args
    import oracle
    import oracle.hamiltonian as oh
    oh._WORKERS = 1
    d = np.load(cache)
    cfg = workloads.get_config(name)
    s = oracle.build_system(name)
    eps, Psi = d["eps"][:cfg.nv], d["psi"][:cfg.nv]
    its = 0
    for j, v in pairs:
        b = oracle.rhs(s, Psi, v, workloads.dv_r(cfg, j))
        _, it, rel, st = oracle.pcg_solve(s, Psi, eps, v, b, tol=tol)
        its += it
    return its


def cpu_baseline(name: str, tol: float, nsample: int):
    """Oracle solves/s on a bounded sample, process pool of single-threaded workers."""
    cfg = workloads.get_config(name)
    cache = os.path.join(ROOT, "tests", "_cache", f"{name}_seed{cfg.seed_kb}_valence.npz")
    if not os.path.exists(cache):
        return None
    import multiprocessing as mp
    cores = min(16, os.cpu_count() or 1)
    nsample = max(cores, nsample - nsample % cores)
    rng = np.random.default_rng(3)
    pairs = [(int(rng.integers(cfg.npert)), int(rng.integers(cfg.nv))) for _ in range(nsample)]
    chunks = [(name, cache, pairs[i::cores], tol) for i in range(cores)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        its = sum(pool.map(_oracle_worker, chunks))
    dt = time.perf_counter() - t0
    return {"value": nsample / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{nsample} random (perturbation, band) solves of {name} at tol {tol:g}, "
                      f"{its} CG iterations in total, {dt:.1f} s wall on {cores} worker processes "
                      f"(one thread each), valence states from the oracle cache"}


# ---------------------------------------------------------------- served mode
def served(args):
    """Poisson stream of solve requests over systems of different grid sizes (one
    ΔV block of 32 perturbations x all bands per request), mixed precision.  The
    arrival rate is 0.7 x the measured saturation request rate; prints one JSON
    line with request and solve latency percentiles."""
    import torch  # noqa: F401  (device runtime of the process)
    import paper_2203_05623_amd as P

    names = args.served_systems.split(",")
    # the 432-band valence set-up of the 96^3 system takes minutes: one progress
    # line per eigensolver iteration
    os.environ.setdefault("STH_VERBOSE", "1")
    ctx = P.sth_create(device=0, max_slots=args.slots)
    systems = {}
    for name in names:
        cfg = workloads.get_config(name)
        miller = workloads.miller_sphere(cfg.M2)
        vloc = workloads.vloc_r(cfg)
        beta = workloads.beta_projectors(cfg, miller)
        dij = workloads.dij(cfg)
        t0 = time.perf_counter()
        eps, psi, res, its = P.sth_valence(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, cfg.nv + 1,
                                           tol=1e-10)
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi[:cfg.nv],
                               eps[:cfg.nv])
        import torch as _t
        dv = _t.from_numpy(workloads.dv_block(cfg, range(cfg.npert))).to("cuda:0")
        systems[name] = dict(cfg=cfg, sid=sid, dv=dv, gap=float(eps[cfg.nv] - eps[cfg.nv - 1]),
                             setup_s=time.perf_counter() - t0)
        print(f"{name}: setup {systems[name]['setup_s']:.1f} s, gap {systems[name]['gap']:.4f} Ha",
              file=sys.stderr, flush=True)
    prec = PRECISIONS[args.precision](P)

    def submit(name):
        s = systems[name]
        return P.sth_submit_solves(ctx, s["sid"], s["dv"], np.arange(s["cfg"].nv), tol=args.tol,
                                   precision=prec)

    rng = np.random.default_rng(4)
    # saturation: a burst of requests, throughput = requests / makespan
    burst = [names[i % len(names)] for i in range(2 * len(names))]
    t0 = time.perf_counter()
    tickets = [submit(n) for n in burst]
    for t in tickets:
        P.sth_wait(ctx, t, 3600.0)
        P.sth_release_ticket(ctx, t)
    sat = len(burst) / (time.perf_counter() - t0)
    rate = 0.7 * sat
    print(f"saturation {sat:.3f} req/s, arrival rate {rate:.3f} req/s", file=sys.stderr, flush=True)
    nreq = args.served_requests
    warm = max(1, nreq // 10)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq + warm))
    choice = rng.integers(len(names), size=nreq + warm)
    live = []
    t_start = time.perf_counter()
    for k in range(nreq + warm):
        now = time.perf_counter() - t_start
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        live.append((k, names[choice[k]], submit(names[choice[k]])))
        if (k + 1) % 10 == 0:
            print(f"submitted {k + 1} of {nreq + warm} requests", file=sys.stderr, flush=True)
    req_lat, solve_lat, done_solves = [], [], 0
    for k, name, t in live:
        P.sth_wait(ctx, t, 3600.0)
        if (k + 1) % 10 == 0:
            print(f"request {k + 1} done", file=sys.stderr, flush=True)
        info = P.sth_poll(ctx, t)
        if k >= warm:
            n = info["n_total"]
            _, _, st, lat = P.sth_fetch_stats(ctx, t, n)
            req_lat.append(info["t_done"] - info["t_submit"])
            solve_lat.append(lat)
            done_solves += n
        P.sth_release_ticket(ctx, t)
    span = time.perf_counter() - t_start
    P.sth_destroy(ctx)
    req_lat = np.array(req_lat) * 1e3
    solve_lat = np.concatenate(solve_lat) * 1e3
    out = {"mode": "served", "systems": {n: {"grid": s["cfg"].N, "bands": s["cfg"].nv,
                                              "npw": len(workloads.miller_sphere(s["cfg"].M2)),
                                              "gap_Ha": s["gap"]} for n, s in systems.items()},
           "precision": args.precision, "tol": args.tol, "requests": nreq, "warmup_requests": warm,
           "saturation_req_per_s": sat, "arrival_rate_req_per_s": rate,
           "solves_per_s": done_solves / span,
           "request_latency_ms": {"p50": float(np.percentile(req_lat, 50)),
                                  "p99": float(np.percentile(req_lat, 99))},
           "solve_latency_ms": {"p50": float(np.percentile(solve_lat, 50)),
                                "p99": float(np.percentile(solve_lat, 99))}}
    print(json.dumps(out))


# ---------------------------------------------------------------- dielectric eigensolver
def pdep_run(args):
    """Lowest eigenpairs of chi_bar0 = v^{1/2} chi0 v^{1/2} by the device Davidson
    (sth_pdep) on one system; prints one JSON line with the wall time, the Davidson
    iterations, the solves it ran and the kernel phases of those solves."""
    import torch  # noqa: F401  (device runtime of the process)
    import paper_2203_05623_amd as P

    cfg = workloads.get_config(args.config)
    miller = workloads.miller_sphere(cfg.M2)
    vloc = workloads.vloc_r(cfg)
    beta = workloads.beta_projectors(cfg, miller)
    dij = workloads.dij(cfg)
    ctx = P.sth_create(device=0, max_slots=args.slots)
    if args.valence_cache and os.path.exists(args.valence_cache):
        d = np.load(args.valence_cache)
        eps, psi = d["eps"], d["psi"]
    else:
        eps, psi, _, _ = P.sth_valence(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, cfg.nv + 1,
                                       tol=1e-10)
        if args.valence_cache:
            np.savez(args.valence_cache, eps=eps, psi=psi, res=0.0, iters=0)
    sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi[:cfg.nv],
                           eps[:cfg.nv])
    prec = PRECISIONS[args.precision](P)
    P.sth_profile(ctx, True)
    t0 = time.perf_counter()
    lam, _, its, res = P.sth_pdep(ctx, sid, cfg.N, args.npdep, tol=args.pdep_tol, maxit=200,
                                  solve_tol=args.tol, precision=prec, want_vectors=False)
    dt = time.perf_counter() - t0
    prof = P.sth_profile_read(ctx)
    P.sth_destroy(ctx)
    kernel_ms = sum(v[0] for v in prof.values())
    out = {"mode": "pdep", "config": args.config, "grid": cfg.N, "bands": cfg.nv,
           "npdep": args.npdep, "precision": args.precision, "solve_tol": args.tol,
           "davidson_tol": args.pdep_tol, "iterations": its, "max_residual": res,
           "seconds": dt, "eigenvalues_lowest": [float(x) for x in lam[:8]],
           "solve_kernel_ms": round(kernel_ms, 1),
           "phases_ms": {k: round(v[0], 1) for k, v in prof.items()}}
    print(json.dumps(out))


# ---------------------------------------------------------------- Lanczos chains
def lanczos_run(args):
    """Batched Lanczos chains (sth_lanczos) of one orbital for --nphi band-limited real
    grid functions, --nsteps steps; prints one JSON line with the wall time per call
    (after one warm-up call) and the H applications per second."""
    import torch  # noqa: F401  (device runtime of the process)
    import paper_2203_05623_amd as P

    cfg = workloads.get_config(args.config)
    miller = workloads.miller_sphere(cfg.M2)
    vloc = workloads.vloc_r(cfg)
    beta = workloads.beta_projectors(cfg, miller)
    dij = workloads.dij(cfg)
    ctx = P.sth_create(device=0, max_slots=args.slots)
    if args.valence_cache and os.path.exists(args.valence_cache):
        d = np.load(args.valence_cache)
        eps, psi = d["eps"], d["psi"]
    else:
        eps, psi, _, _ = P.sth_valence(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, cfg.nv + 1,
                                       tol=1e-10)
        if args.valence_cache:
            np.savez(args.valence_cache, eps=eps, psi=psi, res=0.0, iters=0)
    sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi[:cfg.nv],
                           eps[:cfg.nv])
    # smooth real functions on the grid (perturbation-shaped stand-ins for PDEP vectors)
    phi = workloads.dv_block(cfg, range(args.nphi))
    band = cfg.nv - 1
    P.sth_lanczos(ctx, sid, band, phi, args.nsteps)
    t0 = time.perf_counter()
    a, b, dd, U, br = P.sth_lanczos(ctx, sid, band, phi, args.nsteps)
    dt = time.perf_counter() - t0
    P.sth_destroy(ctx)
    out = {"mode": "lanczos", "config": args.config, "grid": cfg.N, "band": band,
           "chains": args.nphi, "steps": args.nsteps, "seconds": dt,
           "h_applications_per_s": args.nphi * args.nsteps / dt,
           "alpha_first": [float(x) for x in a[0, :4]], "beta_first": [float(x) for x in b[0, :4]]}
    print(json.dumps(out))


# ---------------------------------------------------------------- GPU run
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--npert", type=int, default=0, help="override the perturbation count")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--compare", default="mixed-bf16", choices=sorted(PRECISIONS) + [""],
                    help="also time this precision on the same system (empty: skip)")
    ap.add_argument("--slots", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--valence-cache", default="",
                    help="npz file: load the device LOBPCG states from it if present, else "
                         "compute them on the device and save them there")
    ap.add_argument("--served", action="store_true",
                    help="served mode: Poisson request stream over several systems")
    ap.add_argument("--served-systems", default="cfg4a,cfg4b,cfg4c")
    ap.add_argument("--served-requests", type=int, default=40)
    ap.add_argument("--pdep", action="store_true",
                    help="dielectric eigensolver: lowest eigenpairs of v^1/2 chi0 v^1/2")
    ap.add_argument("--npdep", type=int, default=32)
    ap.add_argument("--pdep-tol", type=float, default=1e-5)
    ap.add_argument("--lanczos", action="store_true",
                    help="batched Lanczos chains of one orbital (--nphi chains, --nsteps steps)")
    ap.add_argument("--nphi", type=int, default=64)
    ap.add_argument("--nsteps", type=int, default=30)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for "
              f"--gpus {args.gpus}); the per-GPU work would be sharded by perturbation.",
              file=sys.stderr)
        sys.exit(2)
    if args.served:
        served(args)
        return
    if args.pdep:
        pdep_run(args)
        return
    if args.lanczos:
        lanczos_run(args)
        return
    cfg = workloads.get_config(args.config)
    npert = args.npert or cfg.npert
    nsolves = npert * cfg.nv

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, args.tol, args.cpu_sample)

    import torch
    import paper_2203_05623_amd as P

    if args.calib_copy:
        # a plain copy kernel of known size: reads and writes 1 GiB each
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    miller = workloads.miller_sphere(cfg.M2)
    vloc = workloads.vloc_r(cfg)
    beta = workloads.beta_projectors(cfg, miller)
    dij = workloads.dij(cfg)
    dv = workloads.dv_block(cfg, range(npert))
    ctx = P.sth_create(device=0, max_slots=args.slots)
    t0 = time.perf_counter()
    if args.valence_cache and os.path.exists(args.valence_cache):
        # states computed by an earlier run of the device LOBPCG (profiling runs)
        d = np.load(args.valence_cache)
        eps, psi, vres, vits = d["eps"], d["psi"], float(d["res"]), int(d["iters"])
    else:
        eps, psi, vres, vits = P.sth_valence(ctx, cfg.L, cfg.N, miller, vloc, beta, dij,
                                             cfg.nv + 1, tol=1e-10)
        if args.valence_cache:
            np.savez(args.valence_cache, eps=eps, psi=psi, res=vres, iters=vits)
    t_val = time.perf_counter() - t0
    gap = float(eps[cfg.nv] - eps[cfg.nv - 1])
    sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi[:cfg.nv],
                           eps[:cfg.nv])
    tinfo = P.sth_system_info_get(ctx, sid)
    tuning = {k: tinfo[k] for k in ("fft_plan_fp64", "plane_kernel_fp64", "zfft_kernel_fp64",
                                    "fft_plan_fp32", "plane_kernel_fp32", "zfft_kernel_fp32",
                                    "gemm_kchunk", "tuned_from_cache")}
    tuning["tune_ms"] = [round(x, 4) for x in tinfo["tune_ms"]]
    prec = PRECISIONS[args.precision](P)
    bands = np.arange(cfg.nv)
    dv = torch.from_numpy(dv).to("cuda:0")      # inputs resident in HBM before timing

    def step():
        t = P.sth_submit_solves(ctx, sid, dv, bands, tol=args.tol, precision=prec)
        if not P.sth_wait(ctx, t, 3600.0):
            raise RuntimeError("step did not finish")
        info = P.sth_poll(ctx, t)
        it, res, st, lat = P.sth_fetch_stats(ctx, t, nsolves)
        _, _, lam = P.sth_chi0_block(ctx, t, npert)
        P.sth_release_ticket(ctx, t)
        return info, it, res, st, lat, lam

    for _ in range(args.warmup):
        step()
        print("warmup step done", file=sys.stderr, flush=True)
    P.sth_profile(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, lats, iters, bad, worst = [], [], [], 0, 0.0
    for k in range(args.steps):
        info, it, res, st, lat, lam = step()
        infos.append(info)
        lats.append(lat)
        iters.append(it)
        bad += int((st != 0).sum())
        worst = max(worst, float(res.max()))
        print(f"step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = P.sth_profile_read(ctx)
    P.sth_profile(ctx, False)
    # the other precision of the metric on the same system and inputs (its own
    # warm-up step captures its graphs), reported beside the primary figure
    compare = None
    if args.compare and args.compare != args.precision:
        prec = PRECISIONS[args.compare](P)
        for _ in range(max(args.warmup, 1)):
            step()
        print(f"{args.compare} warmup step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c_lat, c_its, c_bad, c_worst = [], [], 0, 0.0
        for k in range(args.steps):
            info, it, res, st, lt, _ = step()
            c_lat.append(lt)
            c_its.append(it)
            c_bad += int((st != 0).sum())
            c_worst = max(c_worst, float(res.max()))
            print(f"{args.compare} step {k} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        cdt = time.perf_counter() - t1
        cl = np.concatenate(c_lat) * 1e3
        ci = np.concatenate(c_its)
        compare = {"precision": args.compare, "value": args.steps * nsolves / cdt,
                   "ms_per_step": cdt * 1e3 / args.steps,
                   "latency_ms": {"p50": float(np.percentile(cl, 50)),
                                  "p99": float(np.percentile(cl, 99))},
                   "cg_iterations": {"mean": float(ci.mean()), "max": int(ci.max())},
                   "not_converged": c_bad, "max_true_rel_residual": c_worst}
    P.sth_destroy(ctx)

    lat = np.concatenate(lats) * 1e3
    its = np.concatenate(iters)
    value = args.steps * nsolves / dt
    # dominant kernel phase and its roofline: the projector GEMMs against the
    # MFMA peak, the plane stage (FFT butterflies on the vector ALUs) against the
    # vector ALU peak with the nominal 5 N log2 N flops per transform, the other
    # phases against HBM bandwidth; FP64 peaks for FP64 runs, FP32 for mixed.  In
    # the BF16-mixed form a GEMM phase holds the KB products on BF16 MFMA (each
    # algorithmic complex-FP32 flop issued as three BF16 products: hi hi, hi lo,
    # lo hi) and the P_c projection on FP32 MFMA; its peak is the flop-weighted
    # harmonic blend of BF16 / 3 and FP32 over the KB and valence row counts
    dom = max(prof, key=lambda k: prof[k][0])
    ms, nl, by, fl = prof[dom]
    kind = {"gemm_ah_b": "mfma", "gemm_a_c": "mfma", "plane": "alu"}.get(dom, "hbm")
    if kind == "hbm":
        roof = {"bound": "hbm", "achieved": by / (ms * 1e-3) / 1e9, "peak": MI355X_HBM_GBS,
                "unit": "GB/s"}
    else:
        if args.precision == "fp64":
            peak = MI355X_FP64_TFLOPS
        elif kind == "mfma" and args.precision == "mixed-bf16":
            w_kb = beta.shape[0] / (beta.shape[0] + cfg.nv)
            peak = 1.0 / (w_kb * 3.0 / MI355X_BF16_TFLOPS + (1.0 - w_kb) / MI355X_FP32_TFLOPS)
        else:
            peak = MI355X_FP32_TFLOPS
        roof = {"bound": kind, "achieved": fl / (ms * 1e-3) / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
        if kind == "mfma" and args.precision == "mixed-bf16":
            roof["peak_blend"] = {"bf16_x3_rows": int(beta.shape[0]), "fp32_rows": int(cfg.nv)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counters (calibrated
    # on a 1 GiB copy) as a multiple of the algorithmic bytes, where measured
    ratio = HBM_OVER_ALGORITHMIC.get((dom, args.precision))
    roof["traffic"] = None if ratio is None else ratio * by / max(nl, 1)
    roof["traffic_unit"] = "bytes/launch"
    roof["kernel"] = dom
    roof["avg_launch_us"] = ms * 1e3 / max(nl, 1)
    roof["algorithmic_bytes_per_launch"] = by / max(nl, 1)
    roof["algorithmic_flops_per_launch"] = fl / max(nl, 1)
    phases = {k: {"ms": round(v[0], 3), "launches": v[1],
                  "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None,
                  "TFLOP/s": round(v[3] / (v[0] * 1e-3) / 1e12, 2) if v[0] > 0 and v[3] else None}
              for k, v in prof.items()}
    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32/f64", "mixed-bf16": "bf16x2/f32/f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg.natoms}-atom synthetic crystal, {cfg.N}^3 grid, "
                               f"{len(miller)} plane waves, {cfg.nv} bands, {cfg.nproj} KB "
                               f"projectors, {npert} perturbations = {nsolves} solves/step, "
                               f"tol {args.tol:g}, {args.precision}",
                   "solves_per_step": nsolves, "precision": args.precision, "tol": args.tol},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "cg_iterations": {"mean": float(its.mean()), "max": int(its.max())},
        "not_converged": bad, "max_true_rel_residual": worst,
        "setup": {"valence_s": t_val, "valence_iters": vits, "valence_residual": vres,
                  "gap_Ha": gap},
        "roofline": roof, "phases": phases, "tuning": tuning, "cpu_baseline": cpu,
    }
    if compare is not None:
        compare["speedup_over_" + args.precision] = compare["value"] / value
        out["compare"] = compare
    print(json.dumps(out))


if __name__ == "__main__":
    main()
