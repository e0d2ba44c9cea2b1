"""Throughput benchmark of the batched Sternheimer path on one MI355X.

A step is one pass of the whole hot path over one request: the right-hand
sides -P_c dV_j psi_v, the batched PCG solves of every (perturbation, band)
pair to a true relative residual of 1e-8, the density responses dn_j and the
chi0 block Rayleigh-Ritz.  Workload (default): the 512-atom synthetic cell on
a 144^3 grid (187,511 plane waves, 1024 valence bands from the device
eigensolver, 2048 KB projectors), 4 of its 64 perturbations per step = 4,096
solves, in FP64 and (the `compare` object) BF16-mixed precision, timed alike;
then the 64-atom crystal on a 72^3 grid (256 perturbations x 128 bands =
32,768 solves per step) the same way (the `extra` object).  Both sample the
Brillouin zone at Gamma as the paper's benchmarks do: the valence states are
made real in real space (set-up, untimed) and the projector products run on
half the sphere; --complex runs the general complex form instead.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg5] [--npert 4] [--complex]

Prints one JSON line.  The CPU baseline is the oracle (plain FP64 NumPy PCG)
timed on a bounded sample of the same solves by worker processes forked
before the GPU is touched.
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
# (workload, phase, precision) -> measured HBM bytes / algorithmic bytes of the
# phase's kernels over one run of the same workload (rocprofv3 FETCH_SIZE x2 +
# WRITE_SIZE, summed over every launch of the phase; profiles/ holds the
# summaries and commands); entries are dropped whenever those kernels change
HBM_OVER_ALGORITHMIC = {
    # 144^3: split-K projector GEMM (W and P tiles re-read per row / column tile)
    ("cfg5", "gemm_ah_b", "fp64"): 4.796,
    # 144^3 compact-row plane kernels (FP64; FP32 and FP64 in the mixed form)
    ("cfg5", "plane", "fp64"): 1.914, ("cfg5", "plane", "mixed-bf16"): 1.304,
    # 72^3 single-pass plane kernels (persistent form FP64, workgroup form FP32)
    ("cfg2", "plane", "fp64"): 1.005, ("cfg2", "plane", "mixed-bf16"): 1.009,
    ("cfg2", "gemm_ah_b", "fp64"): 1.852,
    # Gamma-point form: the plane kernels are those of the complex form
    ("cfg5/gamma", "plane", "fp64"): 1.909, ("cfg5/gamma", "plane", "mixed-bf16"): 1.327,
    ("cfg2/gamma", "plane", "fp64"): 1.005, ("cfg2/gamma", "plane", "mixed-bf16"): 1.009,
}
# --precision: FP64 solves; mixed (FP32 inner operator, FP32-MFMA projector
# GEMMs); mixed-bf16 (FP32 inner operator, BF16-MFMA hi/lo projector GEMMs)
PRECISIONS = {"fp64": lambda P: P.STH_FP64, "mixed": lambda P: P.STH_MIXED,
              "mixed-bf16": lambda P: P.STH_MIXED_BF16}


# ---------------------------------------------------------------- CPU baseline (oracle)
# The oracle runs in a process pool forked before the GPU is touched.  One
# worker builds the oracle's system and stores its arrays as .npy files in a
# scratch directory while the parent computes the valence states on the GPU;
# the parent stores those states next to them (the oracle has no eigensolver
# that finishes at these sizes); every worker checks its band's residual
# ||H psi_v - eps_v psi_v|| with the oracle's H before timing its solves.
_ORC = {}


def _oracle_env():
    os.environ["OMP_NUM_THREADS"] = "1"
    import oracle.hamiltonian as oh
    oh._WORKERS = 1


def _oracle_prepare(name, scratch):
    _oracle_env()
    import oracle
    t0 = time.perf_counter()
    s = oracle.build_system(name)
    for k in ("miller", "vloc_r", "beta", "dij"):
        np.save(os.path.join(scratch, k + ".npy"), getattr(s, k))
    return time.perf_counter() - t0


def _oracle_sample(args):
    """Right-hand side plus PCG of (j, v) on the oracle, at most `maxit` iterations."""
    name, scratch, j, v, tol, maxit = args
    _oracle_env()
    import oracle
    cfg = workloads.get_config(name)
    if "sys" not in _ORC:
        ld = lambda k: np.load(os.path.join(scratch, k + ".npy"), mmap_mode="r")  # noqa: E731
        _ORC["sys"] = oracle.System(L=cfg.L, N=cfg.N, miller=np.asarray(ld("miller")),
                                    vloc_r=np.asarray(ld("vloc_r")), beta=ld("beta"),
                                    dij=np.asarray(ld("dij")))
        _ORC["eps"], _ORC["psi"] = np.load(os.path.join(scratch, "eps.npy")), ld("psi")
    s, eps, psi = _ORC["sys"], _ORC["eps"], _ORC["psi"]
    hv = oracle.apply_H(s, np.asarray(psi[v])[None])[0]
    vres = float(np.linalg.norm(hv - eps[v] * psi[v]))
    t0 = time.perf_counter()
    b = oracle.rhs(s, psi, v, workloads.dv_r(cfg, j))
    t1 = time.perf_counter()
    _, it, rel, st = oracle.pcg_solve(s, psi, eps, v, b, tol=tol, maxit=maxit)
    t2 = time.perf_counter()
    return {"rhs_s": t1 - t0, "pcg_s": t2 - t1, "iters": it, "status": st, "valence_res": vres}


class OraclePool:
    """Single-threaded oracle workers, forked at construction (before any GPU call)."""

    def __init__(self, name, cores):
        import multiprocessing as mp
        import tempfile
        self.name, self.cores = name, cores
        # scratch for the oracle's arrays (projectors and valence states, GBs at
        # 144^3): memory-backed /dev/shm when it has room, else the temp dir
        import shutil
        base = None
        if os.path.isdir("/dev/shm") and shutil.disk_usage("/dev/shm").free > (32 << 30):
            base = "/dev/shm"
        self.scratch = tempfile.mkdtemp(prefix="sth_oracle_", dir=base)
        self.pool = mp.get_context("fork").Pool(cores)
        self.prep = self.pool.apply_async(_oracle_prepare, (name, self.scratch))

    def set_valence(self, eps, psi):
        try:
            np.save(os.path.join(self.scratch, "eps.npy"), np.asarray(eps))
            np.save(os.path.join(self.scratch, "psi.npy"), np.asarray(psi))
        except OSError as e:   # scratch space: reported by run()
            self.error = e

    def run(self, npert, nv, tol, nsample, maxit, gpu_mean_iters):
        if getattr(self, "error", None) is not None:
            raise self.error
        build_s = self.prep.get()
        rng = np.random.default_rng(3)
        pairs = [(int(rng.integers(npert)), int(rng.integers(nv))) for _ in range(nsample)]
        t0 = time.perf_counter()
        res = self.pool.map(_oracle_sample, [(self.name, self.scratch, j, v, tol, maxit)
                                             for j, v in pairs], chunksize=1)
        wall = time.perf_counter() - t0
        worst_vres = max(r["valence_res"] for r in res)
        if not worst_vres <= 1e-9:
            raise RuntimeError(f"valence states fail the oracle's residual check ({worst_vres:.2e})")
        its = sum(r["iters"] for r in res)
        full = all(r["status"] == 0 for r in res)
        t_rhs = sum(r["rhs_s"] for r in res) / len(res)
        t_it = sum(r["pcg_s"] for r in res) / its
        if full:   # whole solves: time per solve as measured
            per_solve = t_rhs + t_it * its / len(res)
            how = f"{len(res)} whole solves ({its} PCG iterations)"
        else:      # bounded solves: per-iteration time x the GPU run's mean iteration count
            per_solve = t_rhs + t_it * gpu_mean_iters
            how = (f"{len(res)} solves cut at {maxit} PCG iterations each (right-hand side "
                   f"{t_rhs:.2f} s, {t_it:.2f} s per iteration), extrapolated to "
                   f"{gpu_mean_iters:.1f} iterations per solve (the GPU run's mean)")
        cpu_model = ""
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        return {"value": self.cores / per_solve, "unit": "solves/s", "cores": self.cores,
                "kind": "oracle", "value_1core": 1.0 / per_solve,
                "cpu_model": cpu_model, "os_cpu_count": os.cpu_count(),
                "sample": f"{how} of random (perturbation, band) pairs of {self.name} at tol "
                          f"{tol:g}, {wall:.1f} s wall on {self.cores} worker processes (one "
                          f"thread each); valence states from the GPU run, residual "
                          f"||H psi - eps psi|| <= {worst_vres:.1e} on the oracle's H; oracle "
                          f"system set-up {build_s:.0f} s not timed"}

    def close(self):
        import shutil
        # idle workers leave on their own (no signal: a profiler's handler in a
        # forked worker would report a termination signal as a crash)
        self.pool.close()
        self.pool.join()
        shutil.rmtree(self.scratch, ignore_errors=True)


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
# perturbations per step of the default workloads: the 512-atom share runs 4 of
# its 64 perturbations x 1024 bands per step (4,096 solves, two fills of the
# 2048-slot pool) so that a step stays near half a minute in FP64; the 64-atom
# crystal runs all 256 x 128
DEFAULT_NPERT = {"cfg5": 4}


def _system(cfg):
    miller = workloads.miller_sphere(cfg.M2)
    return (miller, workloads.vloc_r(cfg), workloads.beta_projectors(cfg, miller),
            workloads.dij(cfg))


def _peak(kind, precision, nproj, nv):
    """Peak of a phase: FP64 / FP32 vector ALU or MFMA; for the BF16-mixed GEMM
    phases the flop-weighted harmonic blend of BF16 / 3 (KB rows, three bf16
    products per complex-FP32 flop) and FP32 (valence rows)."""
    if precision == "fp64":
        return MI355X_FP64_TFLOPS
    if kind == "mfma" and precision == "mixed-bf16":
        w_kb = nproj / (nproj + nv)
        return 1.0 / (w_kb * 3.0 / MI355X_BF16_TFLOPS + (1.0 - w_kb) / MI355X_FP32_TFLOPS)
    return MI355X_FP32_TFLOPS


def _roofline(prof, precision, nproj, nv, workload):
    dom = max(prof, key=lambda k: prof[k][0])
    ms, nl, by, fl = prof[dom]
    kind = {"gemm_ah_b": "mfma", "gemm_a_c": "mfma", "plane": "alu"}.get(dom, "hbm")
    if kind == "hbm":
        roof = {"bound": "hbm", "achieved": by / (ms * 1e-3) / 1e9, "peak": MI355X_HBM_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": kind, "achieved": fl / (ms * 1e-3) / 1e12,
                "peak": _peak(kind, precision, nproj, nv), "unit": "TFLOP/s"}
        if kind == "mfma" and precision == "mixed-bf16":
            roof["peak_blend"] = {"bf16_x3_rows": int(nproj), "fp32_rows": int(nv)}
    roof["frac"] = roof["achieved"] / roof["peak"]
    ratio = HBM_OVER_ALGORITHMIC.get((workload, dom, precision))
    roof["traffic"] = None if ratio is None else ratio * by / max(nl, 1)
    roof["traffic_unit"] = "bytes/launch"
    roof["kernel"] = dom
    roof["avg_launch_us"] = ms * 1e3 / max(nl, 1)
    roof["algorithmic_bytes_per_launch"] = by / max(nl, 1)
    roof["algorithmic_flops_per_launch"] = fl / max(nl, 1)
    return roof


def _realify(P, torch, ctx, sid, miller, psi):
    """Set-up of Gamma-point runs (not timed): an orthonormal basis of the
    occupied space whose vectors are real in real space, c(-G) = conj c(G),
    and H's eigenpairs in it.  The occupied space of a real Hamiltonian with a
    gap above it is closed under c -> conj c(-G), so the symmetric and
    antisymmetric parts of the given states span it; the nv largest
    eigenvalues of their real Gram matrix pick the basis and a Rayleigh-Ritz
    step on it (H applied by the library) the rotation.  Products run on the
    GPU in FP64 (torch), the small eigenproblems on the host."""
    nv = psi.shape[0]
    dev = "cuda:0"
    pos = {tuple(m): i for i, m in enumerate(miller.tolist())}
    mir = torch.tensor([pos[(-a, -b, -c)] for a, b, c in miller.tolist()], device=dev)
    ps = torch.from_numpy(np.ascontiguousarray(psi)).to(dev)
    jp = ps[:, mir].conj()
    S = torch.cat([(ps + jp) * 0.5, (ps - jp) * (-0.5j)])
    del ps, jp
    G = (S.conj() @ S.T.contiguous()).real.cpu().numpy()
    w, U = np.linalg.eigh((G + G.T) / 2)
    idx = np.argsort(w)[::-1]
    if not (w[idx[nv - 1]] > 0.5 and w[idx[nv]] < 1e-6):
        raise RuntimeError(f"occupied space not closed under c -> conj c(-G): Gram eigenvalues "
                           f"{w[idx[nv - 1]]:.3e}, {w[idx[nv]]:.3e} around band {nv}")
    R = torch.from_numpy(np.ascontiguousarray(U[:, idx[:nv]].T / np.sqrt(w[idx[:nv]])[:, None]))
    B = R.to(dev, torch.complex128) @ S
    del S
    HB = P.sth_apply_h(ctx, sid, B)
    Hs = (B.conj() @ HB.T.contiguous()).real.cpu().numpy()
    del HB
    e, V = np.linalg.eigh((Hs + Hs.T) / 2)
    out = (torch.from_numpy(np.ascontiguousarray(V.T)).to(dev, torch.complex128) @ B).cpu()
    return e, out.numpy()


def run_workload(P, torch, name, npert, args, pool=None):
    """Valence set-up, resident system, then timed steps of every requested
    precision (profiling off, captured graphs on) and one profiled step of the
    primary precision (per-phase kernel times, not part of the timed figures)."""
    cfg = workloads.get_config(name)
    nsolves = npert * cfg.nv
    miller, vloc, beta, dij = _system(cfg)
    ctx = P.sth_create(device=0, max_slots=args.slots)
    try:
        t0 = time.perf_counter()
        cache = args.valence_cache if name == args.config else ""
        if cache and os.path.exists(cache):
            # states of an earlier run of the device eigensolver (profiling passes)
            d = np.load(cache)
            eps, psi, vres, vits = d["eps"], d["psi"], float(d["res"]), int(d["iters"])
        else:
            eps, psi, vres, vits = P.sth_valence(ctx, cfg.L, cfg.N, miller, vloc, beta, dij,
                                                 cfg.nv + 1, tol=1e-10)
            if cache:
                np.savez(cache, eps=eps, psi=psi, res=vres, iters=vits)
        t_val = time.perf_counter() - t0
        print(f"{name}: valence set-up {t_val:.1f} s ({vits} iterations, residual {vres:.1e})",
              file=sys.stderr, flush=True)
        gap = float(eps[cfg.nv] - eps[cfg.nv - 1])
        t0 = time.perf_counter()
        sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi[:cfg.nv],
                               eps[:cfg.nv])
        t_sys = time.perf_counter() - t0
        if pool is not None:
            pool.set_valence(eps[:cfg.nv], psi[:cfg.nv])
        t_real = None
        gamma = not args.complex
        if gamma:
            # Gamma-point form: states real in real space, projector products on
            # half the sphere
            t0 = time.perf_counter()
            eps_g, psi_g = _realify(P, torch, ctx, sid, miller, psi[:cfg.nv])
            P.sth_release_system(ctx, sid)
            t_real = time.perf_counter() - t0
            print(f"{name}: Gamma-point states in {t_real:.1f} s (max |eps - eps_complex| "
                  f"{np.abs(eps_g - eps[:cfg.nv]).max():.1e})", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            sid = P.sth_set_system(ctx, cfg.L, cfg.N, miller, vloc, beta, dij, psi_g, eps_g,
                                   gamma_only=True)
            t_sys = time.perf_counter() - t0
            del psi_g
        del psi
        tinfo = P.sth_system_info_get(ctx, sid)
        tuning = {k: tinfo[k] for k in ("fft_plan_fp64", "plane_kernel_fp64", "zfft_kernel_fp64",
                                        "fft_plan_fp32", "plane_kernel_fp32", "zfft_kernel_fp32",
                                        "gemm_kchunk", "tuned_from_cache", "nslots")}
        tuning["tune_ms"] = [round(x, 4) for x in tinfo["tune_ms"]]
        bands = np.arange(cfg.nv)
        dv = torch.from_numpy(workloads.dv_block(cfg, range(npert))).to("cuda:0")

        def step(prec):
            t = P.sth_submit_solves(ctx, sid, dv, bands, tol=args.tol, precision=prec)
            # a long step reports its progress every 30 s (solves finished so far)
            t_wait = time.perf_counter()
            while not P.sth_wait(ctx, t, 30.0):
                if time.perf_counter() - t_wait > 3600.0:
                    raise RuntimeError("step did not finish")
                info = P.sth_poll(ctx, t)
                print(f"{name}: {info['n_finished']} of {info['n_total']} solves finished",
                      file=sys.stderr, flush=True)
            it, res, st, lat = P.sth_fetch_stats(ctx, t, nsolves)
            P.sth_chi0_block(ctx, t, npert)
            P.sth_release_ticket(ctx, t)
            return it, res, st, lat

        legs = {}
        for pname in [args.precision] + ([args.compare] if args.compare and
                                         args.compare != args.precision else []):
            prec = PRECISIONS[pname](P)
            for _ in range(args.warmup):
                step(prec)
                print(f"{name} {pname}: warm-up step done", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            mark = time.monotonic_ns()
            t0 = time.perf_counter()
            lats, its, bad, worst = [], [], 0, 0.0
            for k in range(args.steps):
                it, res, st, lat = step(prec)
                lats.append(lat)
                its.append(it)
                bad += int((st != 0).sum())
                worst = max(worst, float(res.max()))
                print(f"{name} {pname}: step {k} done", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            print(f"{name} {pname}: timed window monotonic_ns {mark} {time.monotonic_ns()}",
                  file=sys.stderr, flush=True)
            lat = np.concatenate(lats) * 1e3
            it = np.concatenate(its)
            legs[pname] = {"value": args.steps * nsolves / dt, "ms_per_step": dt * 1e3 / args.steps,
                           "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                          "p99": float(np.percentile(lat, 99))},
                           "cg_iterations": {"mean": float(it.mean()), "max": int(it.max())},
                           "not_converged": bad, "max_true_rel_residual": worst}
        phases = roof = None
        if not args.no_profile_step:
            P.sth_profile(ctx, True)
            step(PRECISIONS[args.precision](P))
            torch.cuda.synchronize()
            prof = P.sth_profile_read(ctx)
            P.sth_profile(ctx, False)
            roof = _roofline(prof, args.precision, beta.shape[0], cfg.nv,
                             name + ("/gamma" if gamma else ""))
            phases = {k: {"ms": round(v[0], 3), "launches": v[1],
                          "GB/s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None,
                          "TFLOP/s": (round(v[3] / (v[0] * 1e-3) / 1e12, 2)
                                      if v[0] > 0 and v[3] else None)}
                      for k, v in prof.items()}
            print(f"{name}: profiled step done", file=sys.stderr, flush=True)
    finally:
        P.sth_destroy(ctx)
    desc = (f"{name}: {cfg.natoms}-atom synthetic crystal, {cfg.N}^3 grid, {len(miller)} plane "
            f"waves, {cfg.nv} bands, {beta.shape[0]} KB projectors; {npert} of the workload's "
            f"{cfg.npert} perturbations x {cfg.nv} bands = {nsolves} solves per step "
            f"(+ Delta n and the chi0 block), tol {args.tol:g} true relative residual"
            + (", Gamma-point states (half-sphere projector products)" if gamma else
               ", general complex form"))
    return {"name": name, "desc": desc, "nsolves": nsolves, "legs": legs, "roofline": roof,
            "phases": phases, "tuning": tuning,
            "setup": {"valence_s": t_val, "valence_iters": vits, "valence_residual": vres,
                      "gap_Ha": gap, "set_system_s": t_sys, "gamma_states_s": t_real}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg5")
    ap.add_argument("--npert", type=int, default=0,
                    help="perturbations per step (default: 4 for cfg5, all otherwise)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    ap.add_argument("--compare", default="mixed-bf16", choices=sorted(PRECISIONS) + [""],
                    help="also time this precision on the same system (empty: skip)")
    ap.add_argument("--extra", default="cfg2",
                    help="second workload timed the same way after the first (empty: skip)")
    ap.add_argument("--slots", type=int, default=2048)
    ap.add_argument("--complex", action="store_true",
                    help="general complex form (projector products over the whole sphere) "
                         "instead of the Gamma-point form of the paper's benchmarks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle solves sampled (0: auto)")
    ap.add_argument("--cpu-maxit", type=int, default=0,
                    help="PCG iterations per sampled oracle solve (0: auto)")
    ap.add_argument("--no-profile-step", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--valence-cache", default="",
                    help="npz file: load the valence states of the main workload (and of the "
                         "pdep / lanczos modes) from it if present, else compute them on the "
                         "device and save them there")
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
    npert = args.npert or DEFAULT_NPERT.get(args.config, cfg.npert)

    pool = None
    if not args.no_cpu_baseline:
        # large systems: each oracle worker holds transient copies of the
        # projector and valence blocks (GBs), so fewer workers there
        big = cfg.N >= 96
        cores = min(8 if big else 16, os.cpu_count() or 1)
        pool = OraclePool(args.config, cores)

    import torch
    import paper_2203_05623_amd as P

    if args.calib_copy:
        # a plain copy kernel of known size: reads and writes 1 GiB each
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    main_run = run_workload(P, torch, args.config, npert, args, pool)
    cpu = None
    if pool is not None:
        big = cfg.N >= 96
        nsample = args.cpu_sample or pool.cores * (1 if big else 2)
        maxit = args.cpu_maxit or (3 if big else 1000)
        try:
            cpu = pool.run(npert, cfg.nv, args.tol, nsample, maxit,
                           main_run["legs"][args.precision]["cg_iterations"]["mean"])
        except (OSError, RuntimeError) as e:   # scratch space, valence check
            print(f"oracle baseline failed: {e}", file=sys.stderr, flush=True)
            cpu = {"value": None, "error": str(e)}
        finally:
            pool.close()
        print("oracle baseline done", file=sys.stderr, flush=True)
    extra = None
    if args.extra and args.extra != args.config:
        ecfg = workloads.get_config(args.extra)
        extra = run_workload(P, torch, args.extra, DEFAULT_NPERT.get(args.extra, ecfg.npert),
                             args, None)

    prim = main_run["legs"][args.precision]
    out = {
        "metric": METRIC, "value": prim["value"], "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32/f64", "mixed-bf16": "bf16x2/f32/f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": main_run["desc"] + f", {args.precision}",
                   "solves_per_step": main_run["nsolves"], "precision": args.precision,
                   "tol": args.tol},
        "latency_ms": prim["latency_ms"], "cg_iterations": prim["cg_iterations"],
        "not_converged": prim["not_converged"],
        "max_true_rel_residual": prim["max_true_rel_residual"],
        "setup": main_run["setup"], "roofline": main_run["roofline"],
        "phases": main_run["phases"], "tuning": main_run["tuning"], "cpu_baseline": cpu,
    }
    if args.compare and args.compare in main_run["legs"] and args.compare != args.precision:
        c = dict(main_run["legs"][args.compare], precision=args.compare)
        c["speedup_over_" + args.precision] = c["value"] / prim["value"]
        out["compare"] = c
    if extra is not None:
        e = {"workload": extra["desc"], "solves_per_step": extra["nsolves"],
             "setup": extra["setup"], "roofline": extra["roofline"]}
        for k, leg in extra["legs"].items():
            e[k] = leg
        out["extra"] = e
    print(json.dumps(out))


if __name__ == "__main__":
    main()
