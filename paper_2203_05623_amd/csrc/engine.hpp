// Host side of the Sternheimer library: resident systems, the solve server
// and its slot pool.  One process, one device per context.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

// split-K of C = W^H P: at most kMaxSplit chunks of K; chunk lengths are
// multiples of the 16-element LDS stage of the GEMM kernel
constexpr int kMaxSplit = 32;

// Forms of the operator A = H - eps + alpha P_v a CG step applies: the FP64
// operator, the FP32 inner operator with FP32-MFMA projector GEMMs, and the FP32
// inner operator with BF16-MFMA (hi/lo) projector GEMMs; index of a solve's
// precision (STH_FP64, STH_MIXED, STH_MIXED_BF16).
enum OpMode : int { OP_FP64 = 0, OP_FP32 = 1, OP_BF16 = 2 };
inline int split_chunk(int K, int nsplit) {
  const int c = (K + nsplit - 1) / nsplit;
  return ((c + 15) / 16) * 16;
}


double now_s();

// Static device work space of the allocation-free entry point (noalloc.cpp):
// its address on the current device is taken once per device at context creation.
void noalloc_init(int device);
size_t noalloc_capacity();

// Owning device allocation, charged against the context's HBM budget.
class Budget;
class DevMem {
 public:
  DevMem() = default;
  DevMem(Budget* b, size_t bytes);
  ~DevMem();
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept { *this = std::move(o); }
  DevMem& operator=(DevMem&& o) noexcept;
  template <typename T>
  T* as() const { return static_cast<T*>(p_); }
  size_t bytes() const { return n_; }
  void zero(hipStream_t st);

 private:
  void release();
  void* p_ = nullptr;
  size_t n_ = 0;
  Budget* b_ = nullptr;
};

class Budget {
 public:
  explicit Budget(size_t limit) : limit_(limit) {}
  void set_limit(size_t limit) { limit_ = limit; }
  bool fits(size_t bytes) const { return used_ + bytes <= limit_; }
  void charge(size_t bytes);   // throws STH_E_NOMEM
  void credit(size_t bytes) { used_ -= bytes; }
  size_t used() const { return used_; }
  size_t limit() const { return limit_; }

 private:
  std::atomic<size_t> used_{0};
  size_t limit_;
};

// Pinned host staging.
class HostMem {
 public:
  HostMem() = default;
  explicit HostMem(size_t bytes);
  ~HostMem();
  HostMem(const HostMem&) = delete;
  HostMem& operator=(const HostMem&) = delete;
  HostMem& operator=(HostMem&& o) noexcept {
    std::swap(p_, o.p_);
    return *this;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p_); }

 private:
  void* p_ = nullptr;
};

// Dense Hermitian eigensolver on the device (Jacobi): A (n x n, row-major,
// destroyed), ascending eigenvalues to host w, eigenvectors as columns of V.
void eig_hermitian_device(Budget* b, z64* A, int n, double* w, z64* V, hipStream_t st);
void small_mm_device(const z64* A, const z64* B, z64* C, int n, bool ah, hipStream_t st);
void scale_cols_device(z64* V, int n, const double* s_dev, hipStream_t st);
// Ascending eigenvalues of the pencil (sym(M), S) of host matrices, on the device.
void gen_eig_device(Budget* b, const std::vector<double>& M, const std::vector<double>& S, int n,
                    double* lam, hipStream_t st);

struct Request;

// A host vector copied into a new device allocation (stream-ordered on st).
template <typename T>
DevMem upload(Budget* b, const std::vector<T>& v, hipStream_t st) {
  DevMem m(b, v.size() * sizeof(T));
  if (!v.empty())
    STH_HIP_CHECK(hipMemcpyAsync(m.as<void>(), v.data(), v.size() * sizeof(T),
                                 hipMemcpyHostToDevice, st));
  return m;
}

// Copies between caller memory (STH_PTR_HOST or STH_PTR_DEVICE) and device memory,
// stream-ordered on st; check_ptr_kind rejects any other kind (STH_E_INVALID).
void copy_in(void* dst, const void* src, size_t bytes, int ptr_kind, hipStream_t st);
void copy_out(void* dst, const void* src, size_t bytes, int ptr_kind, hipStream_t st);
void check_ptr_kind(int k);

// Host-side stick maps of a sphere (see build_sticks).
struct StickBuild {
  std::vector<int> perm;        // caller index -> internal index
  std::vector<int> stick_off, elem_pos, stick_i12, row_list;
  std::vector<double> kin;
};

struct SlotHost {
  Request* req = nullptr;   // owner of the solve in this slot (null = free)
  int solve = -1;           // j * nband + band index within the request
  double t_admit = 0.0;
  int restarts = 0;
};

struct System {
  int id = 0;
  int N = 0, npw = 0, nst = 0, nrow = 0, nv = 0, nproj = 0, M = 0;
  int m2 = 0;          // largest |m|^2 on the sphere (density sphere: |m|^2 <= 4 m2)
  double L = 0.0, omega = 0.0, fs = 2.0;
  GridDev g;
  DevMem d_stick_off, d_elem_pos, d_stick_i12, d_row_list, d_rowbits, d_row_srange, d_kin, d_tw64,
      d_tw32, d_perm;
  DevMem d_stage;      // [kStageSlots][nrow][N] z64 scratch planes of the strip-form kernels
  DevMem d_W;          // [nv + nproj][npw] z64, internal order: psi_v rows, then beta rows
  DevMem d_diag;       // [nv + nproj]: 0 on psi_v rows, D_p on beta rows
  DevMem d_vloc;       // [N^3] double
  DevMem d_W32;        // FP32 copy of W (inner operator of mixed-precision solves)
  DevMem d_Wb;         // bf16 high and low planes of W, rows of bf16_ldw(npw) (STH_MIXED_BF16)
  DevMem d_vloc32;     // FP32 copy of V_loc
  DevMem d_psir;       // [nv][N^3] z64, psi_v(r) without Omega^{-1/2}
  // Gamma-point systems: internal index k0 of G = 0, and for the nmir elements
  // after it the internal index of -G (all before k0)
  bool gamma = false;
  int k0 = 0, nmir = 0;
  DevMem d_mirror;
  DevMem d_eps_band;   // [nv]
  std::vector<double> eps, ekin;   // per band
  std::vector<int> perm;           // caller index -> internal index

  // slot pool
  int nslots = 0;
  int kchunk = 2048, nsplit = 1, ntile = 1, nchunk = 1;
  DevMem d_x, d_r, d_p, d_q, d_b, d_sticks, d_part, d_C, d_dots, d_part2;
  DevMem d_ss_d, d_ss_i;     // SlotState doubles [7][nslots], ints [2][nslots]
  DevMem d_potptr;           // [nslots] const double*
  DevMem d_lists;            // index arena for slot lists
  HostMem h_potptr, h_eps, h_ekin, h_lists, h_status, h_iters, h_rn2, h_bn2;
  SlotState ss;
  std::vector<SlotHost> slots;
  int lists_used = 0;
  DevMem d_drho_sticks;      // [nband_max][N][nst] z64 scratch of the density response
  int drho_nb = 0;

  // hipGraph of `graph_nit` CG iterations over every slot (steady state), one per
  // operator precision; captured on first use, replayed each check period
  double tune_ms[48] = {};         // autotuner timings (see sth_system_info)
  int tuned_from_cache = 0;
  DevMem d_ident;                  // [nslots] 0..nslots-1
  hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
  int graph_nit[3] = {0, 0, 0};
  long long graph_replays = 0;
  ~System() {
    for (auto& gx : graph)
      if (gx) (void)hipGraphExecDestroy(gx);
  }

  size_t resident_bytes = 0;       // device memory of the system and its slot pool
  // value of the context's memory epoch when admission last found no room with
  // nothing of this system running (the server then waits for memory to be freed)
  unsigned long long blocked_epoch = ~0ull;
  std::deque<std::shared_ptr<Request>> waiting;   // submitted, not admitted
  std::vector<std::shared_ptr<Request>> running;  // admitted, unfinished

  VecSet<z64> vec(const DevMem& m) const { return {m.as<z64>(), (long long)npw}; }
  VecSet<const z64> cvec(const DevMem& m) const { return {m.as<const z64>(), (long long)npw}; }
  const z64* W() const { return d_W.as<const z64>(); }
  const z64* beta() const { return d_W.as<const z64>() + (size_t)nv * npw; }
};

struct Request {
  uint64_t ticket = 0;
  int sys_id = 0;
  System* sys = nullptr;
  int npert = 0, nband = 0;
  std::vector<int> bands;
  double tol = 1e-10;
  int maxit = 1000, precision = 0, want_dpsi = 0;
  std::vector<double> dv_host;       // until admission
  DevMem d_dv;                       // [npert][N^3]
  // Delta psi blocks: `win` blocks of [nband][npw] (internal order), one per
  // perturbation in flight.  A request submitted with want_dpsi holds one block
  // per perturbation (block j = perturbation j, kept for fetch_dpsi); otherwise a
  // block returns to the free list once its perturbation's Delta n is formed, so
  // a request of any size streams through a bounded window.
  DevMem d_dpsi;                     // [win][nband][npw]
  int win = 0;
  std::vector<int> blk_of;           // per perturbation: its block, -1 when none
  std::deque<int> free_blk;          // unassigned blocks, handed out in order
  DevMem d_drho;                     // [npert][N^3]
  DevMem d_bands;                    // [nband]
  // progress (guarded by the context mutex)
  int state = 0;                     // 0 queued, 1 running, 2 done, 3 failed
  int next = 0;                      // next solve to assign
  int n_finished = 0, n_converged = 0;
  std::vector<int> pert_left;        // unfinished bands per perturbation
  std::vector<int> drho_pending;     // perturbations whose bands are all finished
  int n_drho_done = 0;
  double max_resid = 0.0, t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  long long cg_its = 0, op_apps = 0, op32_apps = 0;
  std::vector<int> iters, status;
  std::vector<double> resid, latency;
  bool failed = false;
  int fail_code = 0;
};

class Context {
 public:
  Context(const sth_config& cfg);
  ~Context();

  int set_system(const sth_system_desc& d, hipStream_t user);
  void release_system(int id);
  void apply_h(int id, int nvec, const double* in, double* out, int ptr_kind, hipStream_t user);
  void valence(const sth_system_desc& d, int nbands, double tol, int maxit, double* eps_out,
               double* psi_out, int ptr_kind, double* max_resid, int* iters);
  uint64_t submit(int id, int npert, const double* dv, int nband, const int32_t* bands,
                  const sth_solve_opts& o, int ptr_kind, hipStream_t user);
  void poll(uint64_t t, sth_ticket_info* info);
  bool wait(uint64_t t, double timeout);
  void fetch_drho(uint64_t t, double* out, int ptr_kind, hipStream_t user);
  void fetch_dpsi(uint64_t t, double* out, int ptr_kind, hipStream_t user);
  void fetch_stats(uint64_t t, int32_t* iters, double* resid, int32_t* status, double* lat);
  void chi0_block(uint64_t t, double* M, double* S, double* lam);
  void release_ticket(uint64_t t);
  void system_info(int id, sth_system_info* info);
  void pdep(int id, int npdep, int nmax, double tol, int maxit, double solve_tol, int precision,
            double* eig_out, double* vec_out, int ptr_kind, hipStream_t user, int* iters,
            double* max_resid);
  void lanczos(int id, int band, int nphi, const double* phi, int ptr_kind, int nsteps,
               double* alpha, double* beta, double* d, double* U, double* braket,
               hipStream_t user);

 private:
  void autotune(System& s);
  std::shared_ptr<Request> find(uint64_t t);
  System& sys(int id);
  void server_loop();
  bool step(System& s);                       // one check period; true if work was done
  void admit(System& s);
  void refill(System& s);
  void iterate(System& s, const std::vector<int>& act, int nit);
  // one CG iteration (launches only); mode: operator form (OP_FP64, OP_FP32, OP_BF16)
  void cg_step(System& s, const int* dl, int n, int mode);
  void check_and_retire(System& s, std::vector<int>& act);
  void finish_drho(System& s);
  int* upload_list(System& s, const std::vector<int>& v);
  void apply_op(System& s, VecSet<const z64> in, VecSet<z64> out, const int* dl, int n,
                bool dots, int mode = OP_FP64);
  void apply_op32(System& s, VecSet<const z64> in, VecSet<z64> out, const int* dl, int n,
                  bool dots, bool bf16);
  // v <- P_c v on the listed slots (FP64 GEMMs for OP_FP64, FP32 otherwise);
  // with `dots`, partial Re<dot_in, v> per 64-row tile of the projected v into d_dots
  void setup_gamma(System& s, const sth_system_desc& d, const StickBuild& sb);
  // Projector product pair on half the sphere of a Gamma-point system:
  // C = sgn diag (W^H in) (real), out = s0 out + W C, mirrored; with `dots`
  // the tile partials of Re <dot_in, out> over the whole sphere; `phases`
  // books the launches under the GEMM and reduction phases of the profiler
  template <typename T>
  void gamma_pair(System& s, const cpx<T>* A, int M, const double* diag, double sgn,
                  VecSet<const z64> in, VecSet<z64> out, const int* dl, int n, double s0,
                  VecSet<const z64> dot_in, double* dots, cpx<T>* part, cpx<T>* C,
                  bool phases = true);
  void project_c(System& s, VecSet<z64> v, const int* dl, int n, VecSet<const z64> dot_in,
                 bool dots, int mode);
  void order_after(hipStream_t user);   // library stream waits for the user's stream
  void order_before(hipStream_t user);  // user's stream waits for the library stream
  void alloc_slots(System& s, int nslots);
  StickBuild setup_geometry(System& s, const sth_system_desc& d, int nv);
  void validate_desc(const sth_system_desc& d, bool need_psi);
 public:
  // H on a block of device vectors in internal order (no shift): scratch must
  // hold n sticks; used by the valence solver.
  struct HScratch {
    DevMem sticks, part, C, zeros, ids;
    int cap = 0;
  };
  // non-owning view of an H work space (the HScratch buffers, or the static
  // array of the allocation-free entry point)
  struct HView {
    z64 *sticks = nullptr, *part = nullptr, *C = nullptr;
    double* zeros = nullptr;
    int* ids = nullptr;
    int cap = 0;
  };
  void h_block(System& s, HScratch& w, const z64* in, z64* out, int n);
  void h_block_on(System& s, const HView& w, const z64* in, z64* out, int n, hipStream_t st);
  // H c without allocating (work space in a static device array), on `stream`
  void apply_h_noalloc(int id, int nvec, const double* in, double* out, hipStream_t stream);
  void h_scratch(System& s, HScratch& w, int cap);
  Budget* budget() { return &budget_; }
  hipStream_t stream() const { return st_; }

  // kernel timing by phase (HIP events on the library stream)
  enum { PH_ZINV, PH_PLANE, PH_ZFWD, PH_GEMM_AHB, PH_REDUCE, PH_GEMM_AC, PH_CG, PH_OTHER, NPH };
  void profile(bool on);
  void profile_read(double* ms, long long* n, double* bytes, double* flops);
  int prof_begin(int phase);
  void prof_end(int handle, double bytes, double flops);
  void prof_harvest();   // stream must be idle

 private:

  int device_;
  Budget budget_;
  int max_slots_, check_every_, max_queued_;
  bool use_graphs_ = true;
  hipStream_t st_ = nullptr;
  std::mutex mu_;        // tickets, systems map, request progress
  std::mutex gpu_mu_;    // serialises device work of API calls and the server
  std::condition_variable cv_;
  std::thread server_;
  bool stop_ = false;
  std::map<int, std::unique_ptr<System>> systems_;
  std::map<uint64_t, std::shared_ptr<Request>> tickets_;
  int next_sys_ = 1;
  // bumped (under mu_) whenever device memory may have been freed or a request
  // queued: ticket and system releases, submissions
  unsigned long long mem_epoch_ = 0;
  uint64_t next_ticket_ = 1;

  struct ProfRec {
    int phase;
    hipEvent_t a, b;
    double bytes, flops;
  };
  bool prof_on_ = false;
  std::mutex prof_mu_;
  std::vector<ProfRec> prof_recs_;
  std::vector<hipEvent_t> ev_pool_;
  double prof_ms_[NPH] = {}, prof_bytes_[NPH] = {}, prof_flops_[NPH] = {};
  long long prof_n_[NPH] = {};
};

}  // namespace sth
