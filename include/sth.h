/*
 * sth.h -- C-ABI of the MI355X Sternheimer library.
 *
 * The library solves, for a periodic Kohn-Sham system in a plane-wave basis
 * (Gamma point), the linear-response (Sternheimer) equations
 *
 *     P_c (H - eps_v) P_c dpsi_jv = -P_c dV_j psi_v ,   P_c = 1 - sum_v |psi_v><psi_v|
 *
 * for every perturbation dV_j and valence band v of a request, by batched
 * preconditioned conjugate gradient, and returns the density response
 *
 *     dn_j(r) = f_s sum_v [psi_v^*(r) dpsi_jv(r) + c.c.]      ( = chi0 . dV_j )
 *
 * (paper: Section 3, the Sternheimer equation and the density-response
 * equation; P_c = 1 - P_v by completeness; the equations are independent per
 * perturbation, spin and orbital, which the library exploits as batch
 * parallelism).  H = T + V_loc + V_NL is applied by the dual-space technique
 * with sphere-pruned FFTs (Section 4.1) and Kleinman-Bylander projectors.
 *
 * Units: Hartree atomic units.  Cell: cubic, edge L (bohr), FFT grid n^3.
 * Conventions shared by every call:
 *   - plane waves G = (2 pi / L) m for integer Miller indices m; the caller's
 *     order of the npw indices defines the order of every coefficient array;
 *   - psi(r) = Omega^{-1/2} sum_G c(G) exp(i G.r), Omega = L^3;
 *   - real-space arrays are n^3 doubles in C order, element (i0, i1, i2) at
 *     r = (i0, i1, i2) L / n, index (i0 n + i1) n + i2;
 *   - complex arrays are interleaved (re, im) doubles (complex128);
 *   - ptr_kind STH_PTR_HOST: pageable or pinned host memory;
 *     STH_PTR_DEVICE: device memory of the context's GPU (e.g. a torch
 *     tensor's data_ptr()); device inputs are read after all work already
 *     queued on `stream` (a hipStream_t, NULL = default stream), device
 *     outputs are complete before later work on `stream` starts.
 *   - inputs are copied before the call returns; the caller may free them.
 *
 * Errors: every call returns STH_OK (0) or a negative sth_status and sets a
 * thread-local message (sth_last_error).  No exception crosses the ABI.
 * A solve that does not converge is NOT a call error: it is reported per
 * solve by sth_fetch_stats.  All calls are thread-safe.
 */
#ifndef STH_H
#define STH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sth_ctx sth_ctx;

typedef enum {
  STH_OK = 0,
  STH_E_INVALID = -1,   /* bad argument (message says which) */
  STH_E_NOMEM = -2,     /* does not fit the context's HBM budget */
  STH_E_AGAIN = -3,     /* admission queue full, retry later */
  STH_E_NOT_READY = -4, /* ticket not finished */
  STH_E_DEVICE = -5,    /* HIP runtime error */
  STH_E_NOT_FOUND = -6, /* unknown system id or ticket */
  STH_E_INTERNAL = -7
} sth_status;

enum { STH_PTR_HOST = 0, STH_PTR_DEVICE = 1 };

/* Precision of a solve.  STH_FP64: everything in FP64.  STH_MIXED: FP32
 * FFTs / H.psi inside the CG iterations with FP64 recurrences, residuals and
 * P_c; the returned solution always meets tol on the true FP64 residual
 * (paper, Section 4.3 and 5.1: FP32 FFTs and communication, FP64 elsewhere).
 * The Kleinman-Bylander GEMMs of that inner operator run on FP32 MFMA
 * (STH_MIXED) or on BF16 MFMA with FP32 accumulation, each FP32 operand split
 * into a bf16 high and low part (STH_MIXED_BF16); the P_c projection of every
 * inner step runs on FP32 MFMA, that of every FP64 residual on FP64 MFMA. */
enum { STH_FP64 = 0, STH_MIXED = 1, STH_MIXED_BF16 = 2 };

/* Per-solve status codes returned by sth_fetch_stats. */
enum {
  STH_SOLVE_CONVERGED = 0,
  STH_SOLVE_MAXIT = 1,     /* maxit reached; solution is the last iterate */
  STH_SOLVE_BREAKDOWN = 2, /* Re<p, A p> <= 0 (operator not positive definite) */
  STH_SOLVE_NAN = 3        /* non-finite value in the right-hand side or iterates */
};

typedef struct {
  int device;               /* HIP device ordinal */
  size_t hbm_budget_bytes;  /* device memory the context may use; 0 = 90% of free */
  int max_slots;            /* solves in flight per system; 0 = derived from the budget */
  int check_every;          /* CG iterations between convergence polls; 0 = default (2) */
  int max_queued;           /* requests waiting for admission (all systems) before
                               sth_submit_solves returns STH_E_AGAIN; 0 = 1024 */
} sth_config;

typedef struct {
  double L;                 /* cubic cell edge (bohr) */
  int n;                    /* FFT grid points per axis: 24, 48, 72, 96 or 144 */
  int npw;                  /* plane waves in the wave-function sphere */
  const int32_t* miller;    /* [npw][3]; host memory always; must satisfy 4 max|m_i| + 1 <= n */
  const double* vloc_r;     /* [n^3] local potential (Ha) */
  int nproj;                /* Kleinman-Bylander projectors (may be 0) */
  const double* beta;       /* complex128 [nproj][npw] */
  const double* dij;        /* [nproj] KB coefficients (Ha), diagonal */
  int nv;                   /* valence bands (0 allowed only for sth_valence) */
  const double* psi_v;      /* complex128 [nv][npw], orthonormal */
  const double* eps_v;      /* [nv] band energies (Ha), ascending */
  double spin_factor;       /* f_s in dn; 2.0 for a spin-unpolarised system */
  int ptr_kind;             /* of vloc_r, beta, dij, psi_v, eps_v */
  int gamma_only;           /* 1: Gamma-point system (Section 3), every coefficient
                               vector real in real space, c(-G) = conj c(G): the
                               projector products of the solves run on half the
                               sphere (C = 2 Re sum over G = 0 and the half after it,
                               minus the G = 0 term; Y(-G) = conj Y(G)).  The sphere
                               must hold -G with every G, and psi_v and beta must be
                               so symmetric (within 1e-10 of their largest
                               coefficient), else STH_E_INVALID; the right-hand
                               sides are then symmetric since vloc_r and dV are
                               real.  0: general complex vectors. */
} sth_system_desc;

typedef struct {
  double tol;               /* relative true residual ||b - A x|| / ||b|| to reach */
  int maxit;                /* CG iterations per solve (0 = 1000) */
  int precision;            /* STH_FP64, STH_MIXED or STH_MIXED_BF16 */
  int want_dpsi;            /* keep dpsi for sth_fetch_dpsi */
} sth_solve_opts;

typedef struct {
  int state;                /* 0 queued, 1 running, 2 done */
  int n_total;              /* solves in the ticket (npert * nband) */
  int n_finished;           /* solves retired so far */
  int n_converged;          /* of which converged */
  double max_rel_resid;     /* largest final true relative residual so far */
  double t_submit, t_start, t_done;   /* seconds on the library's monotonic clock */
  long long cg_iterations;  /* sum of CG iterations over finished solves */
  long long op_applications;/* operator applications incl. true-residual checks */
  long long op_applications_fp32; /* of which with the FP32 inner operator (mixed forms) */
  long long graph_replays;  /* hipGraph replays of captured CG iterations on the ticket's
                               system so far (steady state with every slot busy) */
  int system_id;            /* system the ticket was submitted to */
  int npert, nband;         /* shape of the request: outputs are [npert][...] */
} sth_ticket_info;

/* Creates a context on cfg->device (cfg may be NULL for defaults).  Starts the
 * context's solve-server thread.  *out is owned by the caller until sth_destroy. */
sth_status sth_create(const sth_config* cfg, sth_ctx** out);

/* Waits for running work, frees every device allocation, joins the server. */
sth_status sth_destroy(sth_ctx* ctx);

/* Uploads one system (paper, Section 4: data is copied to the GPU once and
 * stays resident): validates the sphere (no duplicates, alias-free grid),
 * builds the z-stick maps, keeps V_loc, the projectors, psi_v, eps_v and
 * psi_v(r) on the device.  Fails with STH_E_NOMEM if the resident data plus
 * a minimal slot pool does not fit the budget.  nv >= 1 is required. */
sth_status sth_set_system(sth_ctx* ctx, const sth_system_desc* desc, void* stream,
                          int32_t* system_id);

/* Shape and tuning of a resident system.  The autotuner times, once per system
 * (or reads from the JSON-lines cache named by the environment variable
 * STH_TUNE_CACHE), each combination (radix plan, plane kernel form, z-stick
 * kernel form) of the FFT stages in FP64 and FP32 and the split-K chunk of the
 * projector GEMM on the system's full slot batch, and keeps the fastest. */
typedef struct {
  int npw, nsticks, nslots, nv, nproj;
  int fft_plan_fp64, fft_plan_fp32;   /* 0 or 1: index of the radix factorisation */
  int gemm_kchunk;                    /* split-K chunk of C = W^H P */
  double tune_ms[48];                 /* timings behind the choice, ms per launch set:
                                         [20 p + 10 zkind + 2 kind + plan] for precision p
                                         (0 FP64, 1 FP32), 0 where not timed; [40 + i]
                                         split-K candidate i < 8 (32, 24, 16, 12, 11, 8,
                                         6, 4 chunks, repeats skipped) */
  int tuned_from_cache;
  int plane_kernel_fp64, plane_kernel_fp32;   /* plane kernel form ("kind"): 0 workgroup
                                                 form, 1 wave form (every row / column
                                                 owned by one wavefront), 2 strip form
                                                 (the plane in strips of rows and columns
                                                 through a scratch plane; with 4 the only
                                                 forms of grids above 96, whose plane
                                                 tile exceeds the LDS), 3 persistent
                                                 single-pass form (one workgroup per CU
                                                 walks the planes, loading the next
                                                 plane while transforming one), 4
                                                 compact-row form (only the active rows
                                                 in LDS, every transform in the
                                                 registers of 8 or 16 lanes; any grid
                                                 whose active rows fit the LDS) */
  int zfft_kernel_fp64, zfft_kernel_fp32;     /* z-stick kernel form ("zkind"): 0
                                                 workgroup form, 1 wave form */
  int n;                              /* FFT grid points per axis */
  size_t budget_used, budget_limit;   /* the context's device memory in use (all systems,
                                         slot pools, requests) and its budget, bytes */
} sth_system_info;
sth_status sth_system_info_get(sth_ctx* ctx, int32_t system_id, sth_system_info* info);

/* Frees a system; its unfinished tickets fail with STH_E_NOT_FOUND afterwards. */
sth_status sth_release_system(sth_ctx* ctx, int32_t system_id);

/* out = H c for nvec vectors (complex128 [nvec][npw] in the caller's order);
 * H = T + V_loc + V_NL without shift or projector (dual-space FFT route,
 * Section 4.1).  Synchronous with respect to `stream`. */
sth_status sth_apply_h(sth_ctx* ctx, int32_t system_id, int nvec, const double* in,
                       double* out, int ptr_kind, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same product as
 * sth_apply_h, out = H in for nvec vectors (complex128 [nvec][npw], caller's
 * order), both in DEVICE memory of the context's GPU, enqueued on `stream`
 * (NULL = default stream) without synchronising and without any allocation.
 * The work space is one static device array of 64 MiB per GPU, held until the
 * process ends (vectors are taken in chunks that fit it); a system whose single
 * vector needs more work space than that is refused with STH_E_INVALID.  Every
 * call on a GPU shares the array: calls that overlap on one GPU (different
 * streams, threads or contexts) race and must be ordered by the caller.  The
 * system must stay resident until the enqueued work has run. */
sth_status sth_apply_h_noalloc(sth_ctx* ctx, int32_t system_id, int nvec, const double* in,
                               double* out, void* stream);

/* Lowest nbands eigenpairs of H for a system description whose psi_v / eps_v
 * are ignored (nv may be 0), on the device with FP64 Rayleigh-Ritz: block
 * LOBPCG on nbands + 8 vectors while 3 (nbands + 8) <= 2048, else
 * Chebyshev-filtered subspace iteration (degree 16, Zhou-Saad scaled
 * recurrence, spectrum upper bound from a 12-step Lanczos run) on
 * nbands + max(8, g nbands) vectors, g = 0.4 or the environment variable
 * STH_CHFSI_GUARD; the environment variable STH_VALENCE=lobpcg or chfsi forces
 * one.  Needs 3 (nbands + 8) <= npw
 * (LOBPCG) or 2 nb <= npw (subspace iteration), else STH_E_INVALID.
 * eps_out [nbands], psi_out complex128 [nbands][npw] (caller order), both in
 * `out_ptr_kind` memory.  Converged when every residual ||H x - theta x|| <= tol.
 * *iters and *max_resid report the run.  With the environment variable
 * STH_VERBOSE=1 each iteration prints one progress line (iteration, largest
 * residual, elapsed seconds) to stderr. */
sth_status sth_valence(sth_ctx* ctx, const sth_system_desc* desc, int nbands, double tol,
                       int maxit, double* eps_out, double* psi_out, int out_ptr_kind,
                       double* max_resid, int* iters);

/* Queues npert x nband solves: dV_j = dv_r[j] (real [npert][n^3]) for every
 * band index in bands[0..nband) (0 <= band < nv, no duplicates).  Returns at
 * once with a ticket; the server admits the request when its footprint fits
 * the budget: dV and dn of every perturbation, plus the Delta psi block
 * [nband][npw] of every perturbation when want_dpsi is set, else of a window
 * of perturbations in flight (enough to fill the slot pool, fewer when the
 * budget is short, at least one).  Without want_dpsi a perturbation's block is
 * reused once its dn is formed (in fixed band order), so a request larger than
 * device memory (e.g. 64 perturbations x 1024 bands x 187,511 plane waves,
 * 197 GB of Delta psi) streams through.  STH_E_NOMEM if even the smallest
 * footprint exceeds the whole budget; STH_E_AGAIN if max_queued requests are
 * already waiting for admission (nothing is queued; retry later). */
sth_status sth_submit_solves(sth_ctx* ctx, int32_t system_id, int npert, const double* dv_r,
                             int nband, const int32_t* bands, const sth_solve_opts* opts,
                             int ptr_kind, void* stream, uint64_t* ticket);

/* Non-blocking progress of a ticket. */
sth_status sth_poll(sth_ctx* ctx, uint64_t ticket, sth_ticket_info* info);

/* Blocks until the ticket is done or timeout_s elapses (STH_E_NOT_READY). */
sth_status sth_wait(sth_ctx* ctx, uint64_t ticket, double timeout_s);

/* dn_j(r) for the ticket's perturbations: real [npert][n^3]. */
sth_status sth_fetch_drho(sth_ctx* ctx, uint64_t ticket, double* drho, int ptr_kind,
                          void* stream);

/* dpsi_jv: complex128 [npert][nband][npw] in the caller's coefficient order
 * (requires want_dpsi). */
sth_status sth_fetch_dpsi(sth_ctx* ctx, uint64_t ticket, double* dpsi, int ptr_kind,
                          void* stream);

/* Per-solve results, each array [npert][nband] in host memory (any may be NULL):
 * CG iterations, final true relative residual, STH_SOLVE_* status, latency
 * from admission of the solve to its retirement (s). */
sth_status sth_fetch_stats(sth_ctx* ctx, uint64_t ticket, int32_t* iters, double* rel_resid,
                           int32_t* status, double* latency_s);

/* Rayleigh-Ritz of chi0 in span{dV_j} of a finished ticket (paper, Section 3:
 * the first Rayleigh-Ritz step of the projective eigendecomposition):
 * M_ij = (Omega/n^3) sum_r dV_i dn_j, S_ij = (Omega/n^3) sum_r dV_i dV_j and the
 * ascending eigenvalues of (sym(M), S), computed in FP64 on the device.  Host
 * arrays M, S [npert][npert] and lambda [npert]; any may be NULL. */
sth_status sth_chi0_block(sth_ctx* ctx, uint64_t ticket, double* M, double* S, double* lambda);

/* Frees a finished ticket's device results. */
sth_status sth_release_ticket(sth_ctx* ctx, uint64_t ticket);

/* The npdep lowest (most negative) eigenpairs of chi_bar0 = v^{1/2} chi0 v^{1/2}
 * of a resident system, v^{1/2}(G) = sqrt(4 pi) / |G| (paper, Section 3: the
 * projective dielectric eigendecomposition, whose chi0 products come from the
 * Sternheimer solves).  Block Davidson on real grid functions band-limited to
 * the density sphere |m|^2 <= 4 max|m|^2 of the system's sphere, without G = 0,
 * with the inner product (Omega/n^3) sum_r: each chi_bar0 product runs the
 * Sternheimer solves of every valence band on this context's solve server
 * (true relative residual solve_tol, `precision` STH_FP64 / STH_MIXED /
 * STH_MIXED_BF16); Rayleigh-Ritz in FP64 on the device; the residuals of the
 * unconverged pairs extend the basis (at most nmax >= 2 npdep vectors, then a
 * restart from the Ritz vectors).  Stops when every residual
 * ||chi_bar0 y - lambda y|| <= tol, after maxit iterations, or when no new
 * direction remains.  eig_out [npdep] ascending, host memory; vec_out (may be
 * NULL) real [npdep][n^3] orthonormal eigenvectors (C order) in `vec_ptr_kind`
 * memory; *iters and *max_resid (may be NULL) report the run (max_resid > tol:
 * not converged).  Grids up to 96.  STH_E_INVALID for bad arguments.  With
 * STH_VERBOSE=1 each iteration prints one progress line to stderr. */
sth_status sth_pdep(sth_ctx* ctx, int32_t system_id, int npdep, int nmax, double tol, int maxit,
                    double solve_tol, int precision, double* eig_out, double* vec_out,
                    int vec_ptr_kind, void* stream, int* iters, double* max_resid);

/* Lanczos chains of orbital `band` for nphi real grid functions phi (paper,
 * Section 3, equation "lanczos" and the recurrences before it; Section 4.3 for
 * the braket product).  Chain m starts from u_m = T_S[phi_m psi_band] (product
 * in real space, coefficients on the sphere) and runs nsteps steps of
 *   alpha^l = <q^l|H|q^l>,  r = (H - alpha^l) q^l - beta^l q^{l-1},
 *   r -= sum_{k<=l} <q^k|r> q^k,  beta^{l+1} = ||r||,  q^{l+1} = r / beta^{l+1},
 * q^1 = u_m / ||u_m||, H the FP64 dual-space Hamiltonian of the system.
 * phi: real [nphi][n^3] in `ptr_kind` memory.  Outputs in host memory, row-major:
 * alpha [nphi][nsteps]; beta [nphi][nsteps] with beta[m][0] = ||u_m|| and
 * beta[m][l] (l >= 1) the off-diagonal of the tridiagonal matrix between steps
 * l-1 and l; d [nphi][nsteps] its ascending eigenvalues and U
 * [nphi][nsteps][nsteps] its eigenvectors as columns (d, U may be NULL);
 * braket complex128 [nphi][nphi][nsteps]: <u_n|q^l_m> at [n][m][l] (may be NULL).
 * 1 <= nphi <= 256, 1 <= nsteps <= 200; STH_E_INTERNAL if a chain breaks down. */
sth_status sth_lanczos(sth_ctx* ctx, int32_t system_id, int band, int nphi, const double* phi,
                       int ptr_kind, int nsteps, double* alpha, double* beta, double* d,
                       double* U, double* braket, void* stream);

/* Kernel timing of the solve server, for measurement: with enable != 0 the
 * library records HIP events (on its own stream) around every kernel launch
 * of the CG iterations, grouped by phase:
 *   0 z-stick inverse FFT, 1 plane FFT pass, 2 z-stick forward FFT,
 *   3 projection GEMM C = W^H P, 4 partial-sum reduction, 5 GEMM Y += W C,
 *   6 CG vector kernels, 7 right-hand side and retirement work.
 * sth_profile_read returns, per phase, the summed kernel time (ms), the launch
 * count, and the algorithmic HBM bytes and flops of those launches (the
 * method's minimum traffic / arithmetic, not hardware counters).  Reading
 * resets the counters. */
sth_status sth_profile(sth_ctx* ctx, int enable);
sth_status sth_profile_read(sth_ctx* ctx, double* ms /*[8]*/, long long* launches /*[8]*/,
                            double* bytes /*[8]*/, double* flops /*[8]*/);

/* Message of the last failing call on this thread ("" if none). */
const char* sth_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STH_H */
