// Host side of the Sternheimer library: system setup, the slot pool and the
// solve server that runs the batched preconditioned CG.
//
// Operator (paper, Section 3, the Sternheimer equation): for a solve of band v
//   P_c (H - eps_v) P_c x = b,   b = -P_c (dV_j psi_v),
// with P_c = 1 - sum_v |psi_v><psi_v|.  The CG applies (H - eps_v) (FFT route
// plus the Kleinman-Bylander GEMM pair) to directions kept in range(P_c) and
// projects each result (an FP64 GEMM pair over the psi_v rows of
// W = [psi_v; beta]); P_c (H - eps_v) P_c is positive definite there for a
// band below the gap.  The converged x is projected with P_c once more.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <set>
#include <tuple>

namespace sth {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ memory
void Budget::charge(size_t bytes) {
  size_t cur = used_.load();
  while (true) {
    if (cur + bytes > limit_) {
      set_error("device memory budget exceeded: need %zu more bytes, %zu of %zu in use", bytes,
                cur, limit_);
      throw Error(STH_E_NOMEM);
    }
    if (used_.compare_exchange_weak(cur, cur + bytes)) return;
  }
}

DevMem::DevMem(Budget* b, size_t bytes) : n_(bytes), b_(b) {
  if (bytes == 0) return;
  if (b_) b_->charge(bytes);
  hipError_t e = hipMalloc(&p_, bytes);
  if (e != hipSuccess) {
    if (b_) b_->credit(bytes);
    p_ = nullptr;
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    throw Error(STH_E_NOMEM);
  }
}

void DevMem::release() {
  if (p_) {
    (void)hipFree(p_);
    if (b_) b_->credit(n_);
  }
  p_ = nullptr;
  n_ = 0;
}

DevMem::~DevMem() { release(); }

DevMem& DevMem::operator=(DevMem&& o) noexcept {
  if (this != &o) {
    release();
    p_ = o.p_;
    n_ = o.n_;
    b_ = o.b_;
    o.p_ = nullptr;
    o.n_ = 0;
  }
  return *this;
}

void DevMem::zero(hipStream_t st) {
  if (p_) STH_HIP_CHECK(hipMemsetAsync(p_, 0, n_, st));
}

HostMem::HostMem(size_t bytes) {
  if (bytes == 0) bytes = 8;
  STH_HIP_CHECK(hipHostMalloc(&p_, bytes, hipHostMallocDefault));
  std::memset(p_, 0, bytes);
}
HostMem::~HostMem() {
  if (p_) (void)hipHostFree(p_);
}

namespace {

int imod(int a, int n) { return ((a % n) + n) % n; }

}  // namespace

// Copies `bytes` from caller memory (host or device) into device memory.
void copy_in(void* dst, const void* src, size_t bytes, int ptr_kind, hipStream_t st) {
  if (bytes == 0) return;
  STH_HIP_CHECK(hipMemcpyAsync(dst, src, bytes,
                               ptr_kind == STH_PTR_DEVICE ? hipMemcpyDeviceToDevice
                                                          : hipMemcpyHostToDevice,
                               st));
}

void copy_out(void* dst, const void* src, size_t bytes, int ptr_kind, hipStream_t st) {
  if (bytes == 0) return;
  STH_HIP_CHECK(hipMemcpyAsync(dst, src, bytes,
                               ptr_kind == STH_PTR_DEVICE ? hipMemcpyDeviceToDevice
                                                          : hipMemcpyDeviceToHost,
                               st));
}

void check_ptr_kind(int k) {
  if (k != STH_PTR_HOST && k != STH_PTR_DEVICE) {
    set_error("ptr_kind must be STH_PTR_HOST (0) or STH_PTR_DEVICE (1), got %d", k);
    throw Error(STH_E_INVALID);
  }
}

// ------------------------------------------------------------------ context
Context::Context(const sth_config& cfg)
    : device_(cfg.device), budget_(0), max_slots_(cfg.max_slots),
      check_every_(cfg.check_every > 0 ? cfg.check_every : 2),
      max_queued_(cfg.max_queued > 0 ? cfg.max_queued : 1024) {
  int ndev = 0;
  STH_HIP_CHECK(hipGetDeviceCount(&ndev));
  if (cfg.device < 0 || cfg.device >= ndev) {
    set_error("device %d out of range (%d devices)", cfg.device, ndev);
    throw Error(STH_E_INVALID);
  }
  STH_HIP_CHECK(hipSetDevice(device_));
  size_t fr = 0, tot = 0;
  STH_HIP_CHECK(hipMemGetInfo(&fr, &tot));
  size_t lim = cfg.hbm_budget_bytes ? cfg.hbm_budget_bytes : size_t(0.9 * double(fr));
  budget_.set_limit(lim);
  STH_HIP_CHECK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
  noalloc_init(device_);   // device address of the allocation-free entry point's array
  // STH_GRAPHS=0 turns the captured-iteration replay off (direct launches)
  if (const char* e = std::getenv("STH_GRAPHS")) use_graphs_ = std::atoi(e) != 0;
  server_ = std::thread([this] { server_loop(); });
}

Context::~Context() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (server_.joinable()) server_.join();
  (void)hipSetDevice(device_);
  (void)hipStreamSynchronize(st_);
  tickets_.clear();
  systems_.clear();
  for (auto& r : prof_recs_) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(st_);
}

void Context::order_after(hipStream_t user) {
  hipEvent_t ev;
  STH_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  STH_HIP_CHECK(hipEventRecord(ev, user));
  STH_HIP_CHECK(hipStreamWaitEvent(st_, ev, 0));
  STH_HIP_CHECK(hipEventDestroy(ev));
}

void Context::order_before(hipStream_t user) {
  hipEvent_t ev;
  STH_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  STH_HIP_CHECK(hipEventRecord(ev, st_));
  STH_HIP_CHECK(hipStreamWaitEvent(user, ev, 0));
  STH_HIP_CHECK(hipEventDestroy(ev));
}

System& Context::sys(int id) {
  auto it = systems_.find(id);
  if (it == systems_.end()) {
    set_error("unknown system id %d", id);
    throw Error(STH_E_NOT_FOUND);
  }
  return *it->second;
}

std::shared_ptr<Request> Context::find(uint64_t t) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(t);
  if (it == tickets_.end()) {
    set_error("unknown ticket %llu", (unsigned long long)t);
    throw Error(STH_E_NOT_FOUND);
  }
  return it->second;
}

// ------------------------------------------------------------------ system setup
namespace {

StickBuild build_sticks(const int32_t* mil, int npw, int N, double L) {
  StickBuild s;
  int mmax = 0;
  std::vector<std::tuple<int, int, int, int>> key(npw);
  for (int i = 0; i < npw; ++i) {
    const int a = mil[3 * i], b = mil[3 * i + 1], c = mil[3 * i + 2];
    mmax = std::max({mmax, std::abs(a), std::abs(b), std::abs(c)});
    key[i] = std::make_tuple(b, c, a, i);
  }
  if (4 * mmax + 1 > N) {
    set_error("grid n=%d is not alias-free for the sphere: need 4*max|m|+1 = %d <= n", N,
              4 * mmax + 1);
    throw Error(STH_E_INVALID);
  }
  std::sort(key.begin(), key.end());
  s.perm.resize(npw);
  s.elem_pos.resize(npw);
  s.kin.resize(npw);
  const double bb = 2.0 * M_PI / L;
  int nst = -1, pb = INT32_MIN, pc = INT32_MIN;
  std::set<int> rows;
  for (int k = 0; k < npw; ++k) {
    int b, c, a, i;
    std::tie(b, c, a, i) = key[k];
    if (k > 0) {
      int b0, c0, a0, i0;
      std::tie(b0, c0, a0, i0) = key[k - 1];
      if (b0 == b && c0 == c && a0 == a) {
        set_error("duplicate Miller index (%d, %d, %d)", a, b, c);
        throw Error(STH_E_INVALID);
      }
    }
    if (b != pb || c != pc) {
      ++nst;
      s.stick_off.push_back(k);
      s.stick_i12.push_back(imod(b, N) * N + imod(c, N));
      rows.insert(imod(b, N));
      pb = b;
      pc = c;
    }
    s.perm[i] = k;
    s.elem_pos[k] = nst * N + imod(a, N);
    s.kin[k] = 0.5 * bb * bb * double(a * a + b * b + c * c);
  }
  s.stick_off.push_back(npw);
  s.row_list.assign(rows.begin(), rows.end());
  return s;
}

}  // namespace

void Context::alloc_slots(System& s, int nslots) {
  const int N = s.N;
  s.nslots = nslots;
  const size_t vec = (size_t)nslots * s.npw * sizeof(z64);
  s.d_x = DevMem(&budget_, vec);
  s.d_r = DevMem(&budget_, vec);
  s.d_p = DevMem(&budget_, vec);
  s.d_q = DevMem(&budget_, vec);
  s.d_b = DevMem(&budget_, vec);
  s.d_sticks = DevMem(&budget_, (size_t)nslots * N * s.nst * sizeof(z64));
  const int mrows = std::max(s.M, 1);
  s.d_part = DevMem(&budget_, (size_t)s.nsplit * nslots * mrows * sizeof(z64));
  s.d_C = DevMem(&budget_, (size_t)nslots * mrows * sizeof(z64));
  s.d_dots = DevMem(&budget_, (size_t)nslots * s.ntile * sizeof(double));
  s.d_part2 = DevMem(&budget_, (size_t)nslots * s.nchunk * 2 * sizeof(double));
  s.d_ss_d = DevMem(&budget_, (size_t)9 * nslots * sizeof(double));
  s.d_ss_i = DevMem(&budget_, (size_t)4 * nslots * sizeof(int));
  s.d_ss_d.zero(st_);
  s.d_ss_i.zero(st_);
  double* dd = s.d_ss_d.as<double>();
  int* di = s.d_ss_i.as<int>();
  // rho, bnorm2, rnorm2, alpha, beta, eps, ekin, tol, tgt2 | status, iters, maxit, prec
  s.ss = SlotState{dd, dd + nslots, dd + 2 * nslots, dd + 3 * nslots, dd + 4 * nslots,
                   dd + 5 * nslots, dd + 6 * nslots, dd + 7 * nslots, dd + 8 * nslots,
                   di, di + nslots, di + 2 * nslots, di + 3 * nslots};
  s.d_potptr = DevMem(&budget_, (size_t)nslots * sizeof(double*));
  {
    std::vector<int> id(nslots);
    std::iota(id.begin(), id.end(), 0);
    s.d_ident = upload(&budget_, id, st_);
    STH_HIP_CHECK(hipStreamSynchronize(st_));
  }
  prepare_fft_kernels(s.N);
  const int arena = 16 * nslots + 4 * std::max(s.nv, 1) + 4096;
  s.d_lists = DevMem(&budget_, (size_t)arena * sizeof(int));
  s.h_lists = HostMem((size_t)arena * sizeof(int));
  s.h_potptr = HostMem((size_t)nslots * sizeof(double*));
  // host mirrors of the per-slot constants: eps, ekin, tol (double), maxit, prec (int)
  s.h_eps = HostMem((size_t)nslots * sizeof(double) * 5);
  s.h_status = HostMem((size_t)nslots * sizeof(int) * 2);
  s.h_rn2 = HostMem((size_t)nslots * sizeof(double) * 2);
  s.slots.assign(nslots, SlotHost{});
}

int* Context::upload_list(System& s, const std::vector<int>& v) {
  const int arena = int(s.d_lists.bytes() / sizeof(int));
  if (s.lists_used + (int)v.size() > arena) {
    set_error("internal: slot-list arena overflow");
    throw Error(STH_E_INTERNAL);
  }
  int* h = s.h_lists.as<int>() + s.lists_used;
  int* d = s.d_lists.as<int>() + s.lists_used;
  std::memcpy(h, v.data(), v.size() * sizeof(int));
  STH_HIP_CHECK(hipMemcpyAsync(d, h, v.size() * sizeof(int), hipMemcpyHostToDevice, st_));
  s.lists_used += int(v.size());
  return d;
}

// Gamma-point systems: the internal index k0 of G = 0, the internal index of
// -G for every element after it (the stick-major order puts the sticks of
// negative (m1, m2) and the negative m0 half of the (0, 0) stick before G = 0,
// their mirrors after it), and a check that psi_v and beta are real in real
// space (W(-G) = conj W(G) and Im W(0) = 0 within 1e-10 of the row's largest
// coefficient).
void Context::setup_gamma(System& s, const sth_system_desc& d, const StickBuild& sb) {
  const int npw = s.npw;
  std::vector<int> user_of(npw);
  for (int u = 0; u < npw; ++u) user_of[sb.perm[u]] = u;
  std::map<std::tuple<int, int, int>, int> where;   // Miller index -> internal index
  for (int u = 0; u < npw; ++u) {
    const int* m = d.miller + 3 * u;
    where[std::make_tuple(m[0], m[1], m[2])] = sb.perm[u];
  }
  auto it0 = where.find(std::make_tuple(0, 0, 0));
  if (it0 == where.end()) {
    set_error("gamma_only: the sphere has no G = 0");
    throw Error(STH_E_INVALID);
  }
  s.k0 = it0->second;
  s.nmir = npw - 1 - s.k0;
  if (2 * s.nmir + 1 != npw) {
    set_error("gamma_only: G = 0 at internal index %d of %d: the sphere is not symmetric", s.k0,
              npw);
    throw Error(STH_E_INVALID);
  }
  std::vector<int> mir(s.nmir);
  for (int i = 0; i < s.nmir; ++i) {
    const int* m = d.miller + 3 * user_of[s.k0 + 1 + i];
    auto it = where.find(std::make_tuple(-m[0], -m[1], -m[2]));
    if (it == where.end() || it->second >= s.k0) {
      set_error("gamma_only: -G of (%d, %d, %d) is missing or not before G = 0", m[0], m[1], m[2]);
      throw Error(STH_E_INVALID);
    }
    mir[i] = it->second;
  }
  s.d_mirror = upload(&budget_, mir, st_);
  DevMem out(&budget_, 2 * (size_t)s.M * sizeof(double));
  launch_sym_check(s.d_W.as<z64>(), s.M, npw, s.k0, s.nmir, s.d_mirror.as<int>(),
                   out.as<double>(), st_);
  std::vector<double> h(2 * (size_t)s.M);
  STH_HIP_CHECK(hipMemcpyAsync(h.data(), out.as<void>(), h.size() * sizeof(double),
                               hipMemcpyDeviceToHost, st_));
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  for (int r = 0; r < s.M; ++r)
    if (!(h[r] <= 1e-10 * h[s.M + r])) {
      set_error("gamma_only: %s row %d is not real in real space (|W(-G) - conj W(G)| = %.3g, "
                "largest |W| %.3g)", r < s.nv ? "psi_v" : "beta", r < s.nv ? r : r - s.nv, h[r],
                h[s.M + r]);
      throw Error(STH_E_INVALID);
    }
  s.gamma = true;
}

template <typename T>
void Context::gamma_pair(System& s, const cpx<T>* A, int M, const double* diag, double sgn,
                         VecSet<const z64> in, VecSet<z64> out, const int* dl, int n, double s0,
                         VecSet<const z64> dot_in, double* dots, cpx<T>* part, cpx<T>* C,
                         bool phases) {
  const int k0 = s.k0, Kh = s.npw - k0;
  const double vb = double(Kh) * sizeof(z64), wb = double(Kh) * sizeof(cpx<T>);
  const double gf = 4.0 * M * double(Kh) * n;   // real products over the half sphere
  const int nsp = (Kh + s.kchunk - 1) / s.kchunk;
  // phases == false: the caller books the launches under a phase of its own
  auto begin = [&](int phase) { return phases ? prof_begin(phase) : -1; };
  int h = begin(PH_GEMM_AHB);
  // the projections are real: only Re conj(W) x is formed, and Y += W C takes C real
  launch_gemm_ah_b(A + k0, s.npw, M, VecSet<const z64>{in.base + k0, in.stride}, dl, n, Kh,
                   s.kchunk, part, st_, true);
  prof_end(h, M * wb + n * vb, gf);
  h = begin(PH_REDUCE);
  launch_reduce_parts_gamma<T, cpx<T>>(part, nsp, n, M, diag, sgn, C, A, s.npw, k0, k0, in, dl,
                                       st_);
  prof_end(h, (nsp + 1.0) * n * M * sizeof(cpx<T>), 0.0);
  h = begin(PH_GEMM_AC);
  launch_gemm_a_c(A + k0, s.npw, M, C, VecSet<z64>{out.base + k0, out.stride}, dl, n, Kh, s0,
                  {nullptr, 0}, nullptr, st_, true);
  launch_mirror(out, dl, n, k0, s.nmir, s.d_mirror.as<int>(), st_);
  if (dots)
    launch_dots_tiles(dot_in, {out.base, out.stride}, dl, n, s.npw, s.ntile, dots, st_);
  prof_end(h, M * wb + n * vb * 3.0 + (dots ? n * 2.0 * s.npw * sizeof(z64) : 0.0), gf);
}
template void Context::gamma_pair<double>(System&, const z64*, int, const double*, double,
                                          VecSet<const z64>, VecSet<z64>, const int*, int, double,
                                          VecSet<const z64>, double*, z64*, z64*, bool);
template void Context::gamma_pair<float>(System&, const z32*, int, const double*, double,
                                         VecSet<const z64>, VecSet<z64>, const int*, int, double,
                                         VecSet<const z64>, double*, z32*, z32*, bool);

// Geometry, potentials and W = [psi_v (nv rows, may be 0); beta] of a system on the device.
StickBuild Context::setup_geometry(System& s, const sth_system_desc& d, int nv) {
  s.N = d.n;
  s.npw = d.npw;
  s.nv = nv;
  s.nproj = d.nproj;
  s.M = nv + d.nproj;
  s.L = d.L;
  s.omega = d.L * d.L * d.L;
  s.m2 = 0;
  for (int k = 0; k < d.npw; ++k) {
    const int* m = d.miller + 3 * k;
    s.m2 = std::max(s.m2, m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  }
  s.fs = d.spin_factor;
  StickBuild sb = build_sticks(d.miller, d.npw, d.n, d.L);
  s.nst = int(sb.stick_off.size()) - 1;
  s.nrow = int(sb.row_list.size());
  s.perm = sb.perm;
  const int N = s.N;
  const long long n3 = (long long)N * N * N;

  s.d_stick_off = upload(&budget_, sb.stick_off, st_);
  s.d_elem_pos = upload(&budget_, sb.elem_pos, st_);
  s.d_stick_i12 = upload(&budget_, sb.stick_i12, st_);
  s.d_row_list = upload(&budget_, sb.row_list, st_);
  {
    // two words per row: read only by the tile forms (N <= kTileMaxN)
    std::vector<unsigned long long> bits((size_t)N * 2, 0ull);
    if (N <= 128)
      for (int k = 0; k < s.nst; ++k) {
        const int p = sb.stick_i12[k], i1 = p / N, i2 = p % N;
        bits[2 * i1 + (i2 >> 6)] |= 1ull << (i2 & 63);
      }
    s.d_rowbits = upload(&budget_, bits, st_);
  }
  {
    // stick range of each active row (the sticks are sorted by (m1, m2), so the
    // sticks of one i1 row are contiguous): read by the compact-row form
    std::vector<int> fof(N, -1);
    for (int f = 0; f < s.nrow; ++f) fof[sb.row_list[f]] = f;
    std::vector<int> range((size_t)2 * s.nrow, -1);
    for (int k = 0; k < s.nst; ++k) {
      const int f = fof[sb.stick_i12[k] / N];
      if (range[2 * f] < 0) range[2 * f] = k;
      if (range[2 * f + 1] >= 0 && range[2 * f + 1] != k) {
        set_error("internal: sticks of row %d are not contiguous", sb.row_list[f]);
        throw Error(STH_E_INTERNAL);
      }
      range[2 * f + 1] = k + 1;
    }
    s.d_row_srange = upload(&budget_, range, st_);
  }
  s.d_kin = upload(&budget_, sb.kin, st_);
  s.d_perm = upload(&budget_, sb.perm, st_);
  std::vector<z64> tw64(N);
  std::vector<z32> tw32(N);
  for (int t = 0; t < N; ++t) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * t / N;
    tw64[t] = z64{double(cosl(a)), double(sinl(a))};
    tw32[t] = z32{float(tw64[t].x), float(tw64[t].y)};
  }
  s.d_tw64 = upload(&budget_, tw64, st_);
  s.d_tw32 = upload(&budget_, tw32, st_);
  s.g.N = N;
  s.g.npw = s.npw;
  s.g.nst = s.nst;
  s.g.nrow = s.nrow;
  s.g.stick_off = s.d_stick_off.as<int>();
  s.g.elem_pos = s.d_elem_pos.as<int>();
  s.g.stick_i12 = s.d_stick_i12.as<int>();
  s.g.row_list = s.d_row_list.as<int>();
  s.g.rowbits = s.d_rowbits.as<unsigned long long>();
  s.g.row_srange = s.d_row_srange.as<int>();
  for (int r : sb.row_list) s.g.rowmask[r >> 6] |= 1ull << (r & 63);
  s.g.kin = s.d_kin.as<double>();
  s.g.tw64 = s.d_tw64.as<z64>();
  s.g.tw32 = s.d_tw32.as<z32>();
  // scratch planes of the strip-form plane kernels (sized for FP64)
  s.d_stage = DevMem(&budget_, (size_t)kStageSlots * s.nrow * N * sizeof(z64));
  s.g.stage = s.d_stage.as<void>();
  s.g.stage_slots = kStageSlots;
  // before (or without) the autotuner, grids whose plane tile exceeds the LDS
  // take the compact-row form where its rows fit (the valence set-up runs here)
  for (int k = 0; k < 2; ++k)
    if (N > kTileMaxN && plane_kind_available(s.g, kPlaneRows, k == 1))
      s.g.plane_kind[k] = kPlaneRows;
  prepare_fft_kernels(N);
  // split-K chunk of C = W^H P: the smallest candidate of the autotuner (at most
  // kMaxSplit chunks, a multiple of the 16-element LDS stage); the partial
  // buffer is sized for it
  s.kchunk = split_chunk(s.npw, kMaxSplit);
  s.nsplit = (s.npw + s.kchunk - 1) / s.kchunk;
  s.ntile = gemm_a_c_tiles(s.npw);
  s.nchunk = cg_chunks(s.npw);

  // W = [psi_v; beta] in internal order, diag = [0 on psi_v rows; D]
  s.d_W = DevMem(&budget_, (size_t)s.M * s.npw * sizeof(z64));
  {
    DevMem tmp(&budget_, (size_t)std::max({s.nv, s.nproj, 1}) * s.npw * sizeof(z64));
    if (s.nv) {
      copy_in(tmp.as<void>(), d.psi_v, (size_t)s.nv * s.npw * sizeof(z64), d.ptr_kind, st_);
      launch_permute_in(tmp.as<z64>(), s.npw, s.d_W.as<z64>(), s.npw, s.d_perm.as<int>(), s.npw,
                        s.nv, st_);
    }
    if (s.nproj) {
      copy_in(tmp.as<void>(), d.beta, (size_t)s.nproj * s.npw * sizeof(z64), d.ptr_kind, st_);
      launch_permute_in(tmp.as<z64>(), s.npw, s.d_W.as<z64>() + (size_t)s.nv * s.npw, s.npw,
                        s.d_perm.as<int>(), s.npw, s.nproj, st_);
    }
    STH_HIP_CHECK(hipStreamSynchronize(st_));
  }
  if (d.gamma_only) setup_gamma(s, d, sb);
  std::vector<double> diag(s.M, 0.0);
  if (s.nproj) {
    std::vector<double> dij(s.nproj);
    if (d.ptr_kind == STH_PTR_DEVICE)
      STH_HIP_CHECK(
          hipMemcpy(dij.data(), d.dij, s.nproj * sizeof(double), hipMemcpyDeviceToHost));
    else
      std::memcpy(dij.data(), d.dij, s.nproj * sizeof(double));
    std::copy(dij.begin(), dij.end(), diag.begin() + s.nv);
  }
  s.d_diag = upload(&budget_, diag, st_);
  s.d_vloc = DevMem(&budget_, n3 * sizeof(double));
  copy_in(s.d_vloc.as<void>(), d.vloc_r, n3 * sizeof(double), d.ptr_kind, st_);
  // FP32 copies for the inner operator of mixed-precision solves (rounded once)
  s.d_W32 = DevMem(&budget_, (size_t)s.M * s.npw * sizeof(z32));
  launch_z64_to_z32(s.d_W.as<z64>(), s.d_W32.as<z32>(), (long long)s.M * s.npw, st_);
  s.d_Wb = DevMem(&budget_, 2 * (size_t)s.M * bf16_ldw(s.npw) * sizeof(bz));
  launch_split_w(s.d_W32.as<z32>(), s.M, s.npw, bf16_ldw(s.npw), s.d_Wb.as<bz>(), st_);
  s.d_vloc32 = DevMem(&budget_, n3 * sizeof(float));
  launch_to_f32(s.d_vloc.as<double>(), s.d_vloc32.as<float>(), n3, st_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  return sb;
}

int Context::set_system(const sth_system_desc& d, hipStream_t user) {
  check_ptr_kind(d.ptr_kind);
  if (!(d.L > 0) || d.npw <= 0 || !d.miller || !d.vloc_r || d.nv < 1 || !d.psi_v || !d.eps_v ||
      d.nproj < 0 || (d.nproj > 0 && (!d.beta || !d.dij)) || d.nv >= d.npw) {
    set_error("invalid system description (L, npw, miller, vloc_r, nv>=1, psi_v, eps_v, "
              "beta/dij when nproj>0, nv < npw)");
    throw Error(STH_E_INVALID);
  }
  if (d.n != 24 && d.n != 48 && d.n != 72 && d.n != 96 && d.n != 144) {
    set_error("unsupported grid n=%d (supported: 24, 48, 72, 96, 144)", d.n);
    throw Error(STH_E_INVALID);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  order_after(user);
  const size_t used0 = budget_.used();   // every allocation is made under gpu_mu_
  auto sp = std::make_unique<System>();
  System& s = *sp;
  // host copies of the small per-band inputs
  std::vector<double> eps(d.nv);
  if (d.ptr_kind == STH_PTR_DEVICE)
    STH_HIP_CHECK(hipMemcpy(eps.data(), d.eps_v, d.nv * sizeof(double), hipMemcpyDeviceToHost));
  else
    std::memcpy(eps.data(), d.eps_v, d.nv * sizeof(double));
  for (int v = 1; v < d.nv; ++v)
    if (!(eps[v] >= eps[v - 1])) {
      set_error("eps_v must be ascending (band %d)", v);
      throw Error(STH_E_INVALID);
    }
  s.eps = eps;
  StickBuild sb = setup_geometry(s, d, d.nv);
  const int N = s.N;
  const long long n3 = (long long)N * N * N;
  s.d_eps_band = upload(&budget_, eps, st_);

  // slot pool
  const size_t per_slot = (size_t)5 * s.npw * 16 + (size_t)N * s.nst * 16 +
                          (size_t)s.M * 16 * (1 + (s.npw + 2047) / 2048) + 64 * 8;
  int ns = max_slots_ > 0 ? max_slots_ : 1024;
  const size_t resident = (size_t)s.nv * n3 * 16 + (size_t)s.nv * N * s.nst * 16;
  while (ns > 64 && !budget_.fits(resident + (size_t)ns * per_slot + (budget_.limit() / 4)))
    ns /= 2;
  alloc_slots(s, ns);
  autotune(s);

  // orthonormality of psi_v on the device: G = Psi^H Psi
  {
    std::vector<int> idx(s.nv);
    std::iota(idx.begin(), idx.end(), 0);
    double worst = 0.0;
    for (int c0 = 0; c0 < s.nv; c0 += s.nslots) {
      const int nc = std::min(s.nslots, s.nv - c0);
      std::vector<int> sub(idx.begin() + c0, idx.begin() + c0 + nc);
      s.lists_used = 0;
      int* dl = upload_list(s, sub);
      launch_gemm_ah_b(s.W(), s.npw, s.nv, {s.W(), (long long)s.npw}, dl, nc, s.npw, s.kchunk,
                       s.d_part.as<z64>(), st_);
      launch_reduce_parts(s.d_part.as<z64>(), s.nsplit, nc, s.nv, nullptr, 1.0, s.d_C.as<z64>(),
                          st_);
      std::vector<z64> G((size_t)nc * s.nv);
      STH_HIP_CHECK(hipMemcpyAsync(G.data(), s.d_C.as<void>(), G.size() * sizeof(z64),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      for (int c = 0; c < nc; ++c)
        for (int m = 0; m < s.nv; ++m) {
          const z64 v = G[(size_t)c * s.nv + m];
          const double t = (m == c0 + c) ? 1.0 : 0.0;
          worst = std::max(worst, std::hypot(v.x - t, v.y));
        }
    }
    if (!(worst <= 1e-8)) {
      set_error("psi_v is not orthonormal: max |Psi^H Psi - I| = %.3e", worst);
      throw Error(STH_E_INVALID);
    }
  }
  // kinetic energy per band (preconditioner): sum_G T(G) |psi_v(G)|^2 on the host
  {
    std::vector<z64> W((size_t)s.nv * s.npw);
    STH_HIP_CHECK(hipMemcpyAsync(W.data(), s.d_W.as<void>(), W.size() * sizeof(z64),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    s.ekin.assign(s.nv, 0.0);
    for (int v = 0; v < s.nv; ++v) {
      double e = 0.0;
      for (int k = 0; k < s.npw; ++k) {
        const z64 c = W[(size_t)v * s.npw + k];
        e += sb.kin[k] * (c.x * c.x + c.y * c.y);
      }
      s.ekin[v] = e;
    }
  }
  // psi_v(r) resident (density response): copy rows of Psi into the p pool,
  // inverse FFT to sticks, planes to the full grid
  s.d_psir = DevMem(&budget_, (size_t)s.nv * n3 * sizeof(z64));
  for (int c0 = 0; c0 < s.nv; c0 += s.nslots) {
    const int nc = std::min(s.nslots, s.nv - c0);
    std::vector<int> sub(nc), id(nc);
    std::iota(sub.begin(), sub.end(), c0);
    std::iota(id.begin(), id.end(), 0);
    s.lists_used = 0;
    int* dsrc = upload_list(s, sub);
    int* did = upload_list(s, id);
    VecSet<z64> sticks{s.d_sticks.as<z64>(), (long long)N * s.nst};
    launch_copy_vecs({s.W(), (long long)s.npw}, s.vec(s.d_p), dsrc, did, nc, s.npw, st_);
    launch_zfft_inv<double, z64>(s.g, s.cvec(s.d_p), sticks, did, nc, st_);
    launch_plane_to_grid<double>(s.g, {sticks.base, sticks.stride},
                                 {s.d_psir.as<z64>() + (size_t)c0 * n3, n3}, did, nc, st_);
    STH_HIP_CHECK(hipStreamSynchronize(st_));
  }
  s.drho_nb = s.nv;
  s.d_drho_sticks = DevMem(&budget_, (size_t)s.nv * N * s.nst * sizeof(z64));
  STH_HIP_CHECK(hipStreamSynchronize(st_));

  s.resident_bytes = budget_.used() - used0;
  std::lock_guard<std::mutex> lk(mu_);
  s.id = next_sys_++;
  const int id = s.id;
  systems_[id] = std::move(sp);
  return id;
}

void Context::release_system(int id) {
  std::lock_guard<std::mutex> glk(gpu_mu_);
  std::lock_guard<std::mutex> lk(mu_);
  auto it = systems_.find(id);
  if (it == systems_.end()) {
    set_error("unknown system id %d", id);
    throw Error(STH_E_NOT_FOUND);
  }
  for (auto& kv : tickets_)
    if (kv.second->sys_id == id && kv.second->state < 2) {
      kv.second->state = 3;
      kv.second->failed = true;
      kv.second->fail_code = STH_E_NOT_FOUND;
    }
  (void)hipStreamSynchronize(st_);
  systems_.erase(it);
  ++mem_epoch_;
  cv_.notify_all();
}

// ------------------------------------------------------------------ operator
// Nominal arithmetic of the plane stage for n vectors: per plane, inverse and
// forward length-N transforms along i2 on the active rows and along i1 on all
// columns, 5 N log2 N flops each (the usual FFT count), and the real potential
// multiply (2 flops per point).
static double plane_flops(const System& s, int n) {
  const double N = s.N;
  const double per_fft = 5.0 * N * std::log2(N);
  return double(n) * N * ((2.0 * s.nrow + 2.0 * N) * per_fft + 2.0 * N * N);
}

// out = (H - eps_slot) in, on the listed vectors (slot pool scratch: sticks,
// part, C): the FFT route for T + V_loc and the KB projector GEMMs
// beta D beta^H in.  With `dots`, partial Re<in, out> per 64-row tile.  The CG
// applies it to directions in range(P_c) and projects the result (project_c),
// so that it runs on P_c (H - eps_v) P_c.
void Context::apply_op(System& s, VecSet<const z64> in, VecSet<z64> out, const int* dl, int n,
                       bool dots, int mode) {
  if (mode != OP_FP64) {
    apply_op32(s, in, out, dl, n, dots, mode == OP_BF16);
    return;
  }
  const int N = s.N, M = s.nproj;
  const double z = sizeof(z64), vb = double(s.npw) * z, sb = double(N) * s.nst * z;
  const double gf = 8.0 * M * double(s.npw) * n;
  const double* dkb = s.d_diag.as<double>() + s.nv;
  VecSet<z64> sticks{s.d_sticks.as<z64>(), (long long)N * s.nst};
  int h = prof_begin(PH_ZINV);
  launch_zfft_inv<double, z64>(s.g, in, sticks, dl, n, st_);
  prof_end(h, n * (vb + sb), 0.0);
  h = prof_begin(PH_PLANE);
  launch_plane_local<double>(s.g, sticks, dl, n, s.d_vloc.as<double>(), nullptr, st_);
  prof_end(h, n * 2.0 * sb + double(N) * N * N * 8.0, plane_flops(s, n));
  h = prof_begin(PH_ZFWD);
  launch_zfft_fwd<double, z64>(s.g, {sticks.base, sticks.stride}, out, dl, n, ZF_SHIFT, in,
                               s.ss.eps, st_);
  prof_end(h, n * (sb + 2.0 * vb) + s.npw * 8.0, 0.0);
  if (s.gamma) {
    gamma_pair<double>(s, s.beta(), M, dkb, 1.0, in, out, dl, n, 1.0, in,
                       dots ? s.d_dots.as<double>() : nullptr, s.d_part.as<z64>(),
                       s.d_C.as<z64>());
    return;
  }
  // the GEMM partials are indexed by list position; the slot list maps them back
  h = prof_begin(PH_GEMM_AHB);
  launch_gemm_ah_b(s.beta(), s.npw, M, in, dl, n, s.npw, s.kchunk, s.d_part.as<z64>(), st_);
  prof_end(h, M * vb + n * vb, gf);
  h = prof_begin(PH_REDUCE);
  launch_reduce_parts(s.d_part.as<z64>(), s.nsplit, n, M, dkb, 1.0, s.d_C.as<z64>(), st_);
  prof_end(h, (s.nsplit + 1.0) * n * M * z, 0.0);
  h = prof_begin(PH_GEMM_AC);
  launch_gemm_a_c(s.beta(), s.npw, M, s.d_C.as<z64>(), out, dl, n, s.npw, 1.0, in,
                  dots ? s.d_dots.as<double>() : nullptr, st_);
  prof_end(h, M * vb + n * vb * (dots ? 3.0 : 2.0), gf);
}

// The same operator with the FFT passes, V_loc and the projector GEMMs in FP32
// (inner iterations of mixed-precision solves); the kinetic and eps terms and
// every vector in memory stay FP64.
void Context::apply_op32(System& s, VecSet<const z64> in, VecSet<z64> out, const int* dl, int n,
                         bool dots, bool bf16) {
  const int N = s.N, M = s.nproj;
  const double vb = double(s.npw) * sizeof(z64), sb = double(N) * s.nst * sizeof(z32);
  const double gf = 8.0 * M * double(s.npw) * n;
  const double* dkb = s.d_diag.as<double>() + s.nv;
  const int ldw = bf16_ldw(s.npw);
  const bz* wb = s.d_Wb.as<bz>() + (size_t)s.nv * ldw;   // KB rows of the hi plane
  const long long wplane = (long long)s.M * ldw;
  const z32* w32 = s.d_W32.as<z32>() + (size_t)s.nv * s.npw;
  VecSet<z32> sticks{reinterpret_cast<z32*>(s.d_sticks.as<z64>()), (long long)N * s.nst};
  z32* part = reinterpret_cast<z32*>(s.d_part.as<z64>());
  z32* C = reinterpret_cast<z32*>(s.d_C.as<z64>());
  int h = prof_begin(PH_ZINV);
  launch_zfft_inv<float, z64>(s.g, in, sticks, dl, n, st_);
  prof_end(h, n * (vb + sb), 0.0);
  h = prof_begin(PH_PLANE);
  launch_plane_local<float>(s.g, sticks, dl, n, s.d_vloc32.as<float>(), nullptr, st_);
  prof_end(h, n * 2.0 * sb + double(N) * N * N * 4.0, plane_flops(s, n));
  h = prof_begin(PH_ZFWD);
  launch_zfft_fwd<float, z64>(s.g, {sticks.base, sticks.stride}, out, dl, n, ZF_SHIFT, in,
                              s.ss.eps, st_);
  prof_end(h, n * (sb + 2.0 * vb) + s.npw * 8.0, 0.0);
  if (s.gamma && !bf16) {
    gamma_pair<float>(s, w32, M, dkb, 1.0, in, out, dl, n, 1.0, in,
                      dots ? s.d_dots.as<double>() : nullptr, part, C);
    return;
  }
  // the stick buffer is free once the forward z-FFTs have read it: it holds
  // the bf16 split of the vectors, then of C
  bz* split_scratch = reinterpret_cast<bz*>(s.d_sticks.as<z64>());
  const size_t split_bytes = s.d_sticks.bytes();
  if (s.gamma) {
    // half-sphere products from the 16-byte aligned column kh <= k0 on (the
    // planes are read in 4-column chunks); the reduction removes the doubled
    // columns [kh, k0)
    const int kh = s.k0 & ~3, Kh = s.npw - kh;
    const int nsp = (Kh + s.kchunk - 1) / s.kchunk;
    const double vh = double(Kh) * sizeof(z64), gh = 8.0 * M * double(Kh) * n;
    h = prof_begin(PH_GEMM_AHB);
    launch_gemm_ah_b_bf16(wb, wplane, ldw, kh, M, {in.base + kh, in.stride}, dl, n, Kh,
                          s.kchunk, part, split_scratch, split_bytes, st_);
    prof_end(h, M * vh / 2 + n * vh, gh);
    h = prof_begin(PH_REDUCE);
    launch_reduce_parts_gamma<float, z32>(part, nsp, n, M, dkb, 1.0, C, w32, s.npw, s.k0, kh, in,
                                          dl, st_);
    prof_end(h, (nsp + 1.0) * n * M * sizeof(z32), 0.0);
    h = prof_begin(PH_GEMM_AC);
    launch_gemm_a_c_bf16(wb, wplane, ldw, kh, M, C, {out.base + kh, out.stride}, dl, n, Kh, 1.0,
                         {nullptr, 0}, nullptr, split_scratch, split_bytes, st_);
    launch_mirror(out, dl, n, s.k0, s.nmir, s.d_mirror.as<int>(), st_);
    if (dots)
      launch_dots_tiles(in, {out.base, out.stride}, dl, n, s.npw, s.ntile, s.d_dots.as<double>(),
                        st_);
    prof_end(h, M * vh / 2 + n * vh * 3.0 + (dots ? n * 2.0 * vb : 0.0), gh);
    return;
  }
  h = prof_begin(PH_GEMM_AHB);
  if (bf16)
    launch_gemm_ah_b_bf16(wb, wplane, ldw, 0, M, in, dl, n, s.npw, s.kchunk, part,
                          split_scratch, split_bytes, st_);
  else
    launch_gemm_ah_b(w32, s.npw, M, in, dl, n, s.npw, s.kchunk, part, st_);
  prof_end(h, M * vb / 2 + n * vb, gf);
  h = prof_begin(PH_REDUCE);
  launch_reduce_parts(part, s.nsplit, n, M, dkb, 1.0, C, st_);
  prof_end(h, (s.nsplit + 1.0) * n * M * sizeof(z32), 0.0);
  h = prof_begin(PH_GEMM_AC);
  if (bf16)
    launch_gemm_a_c_bf16(wb, wplane, ldw, 0, M, C, out, dl, n, s.npw, 1.0, in,
                         dots ? s.d_dots.as<double>() : nullptr, split_scratch, split_bytes,
                         st_);
  else
    launch_gemm_a_c(w32, s.npw, M, C, out, dl, n, s.npw, 1.0, in,
                    dots ? s.d_dots.as<double>() : nullptr, st_);
  prof_end(h, M * vb / 2 + n * vb * (dots ? 3.0 : 2.0), gf);
}

// Projection onto the conduction space, q <- q - Psi (Psi^H q), on the
// operator output q = (H - eps_v) p of every CG step and true residual.  The
// CG then runs on P_c (H - eps_v) P_c as the equation of Section 3 states it:
// r stays in range(P_c), rho = <r, K r> = <r, P_c K r>, and the P_c part of
// p = K r + beta p evolves exactly as the direction of a CG preconditioned by
// P_c K P_c.  The P_v part of p is never used: P_c (H - eps_v) maps it to zero
// (Psi are eigenvectors of H), the step length takes <p, P_c q> (partials in
// `dots` with `dot_in` = p), and x's P_v part is removed before every true
// residual and when the solve retires.  The projection must not be skipped in
// mixed solves: the FP32 / BF16 operator leaks a P_v part into q that the
// directions would never remove from r, stalling the inner runs.  Their inner
// steps project with FP32 GEMMs (mode != OP_FP64), which leaves ~1e-7 of
// Psi^H q, a small vector since K is close to 1 where the valence states live;
// FP64 steps and every true residual project in FP64.  (The alternative, a
// shifted operator H - eps_v + alpha P_v on the whole sphere with K applied
// unprojected, needs no projection but about 40% more iterations: K mixes P_v
// components into the CG's spectrum.)
void Context::project_c(System& s, VecSet<z64> v, const int* dl, int n, VecSet<const z64> dot_in,
                        bool dots, int mode) {
  const double vb = double(s.npw) * sizeof(z64);
  const double gf = 8.0 * s.nv * double(s.npw) * n;
  double* dd = dots ? s.d_dots.as<double>() : nullptr;
  if (s.gamma) {
    if (mode == OP_FP64)
      gamma_pair<double>(s, s.W(), s.nv, nullptr, -1.0, {v.base, v.stride}, v, dl, n, 1.0,
                         dot_in, dd, s.d_part.as<z64>(), s.d_C.as<z64>());
    else
      gamma_pair<float>(s, s.d_W32.as<z32>(), s.nv, nullptr, -1.0, {v.base, v.stride}, v, dl, n,
                        1.0, dot_in, dd, reinterpret_cast<z32*>(s.d_part.as<z64>()),
                        reinterpret_cast<z32*>(s.d_C.as<z64>()));
    return;
  }
  int h = prof_begin(PH_GEMM_AHB);
  if (mode == OP_FP64) {
    launch_gemm_ah_b(s.W(), s.npw, s.nv, {v.base, v.stride}, dl, n, s.npw, s.kchunk,
                     s.d_part.as<z64>(), st_);
    prof_end(h, s.nv * vb + n * vb, gf);
    h = prof_begin(PH_REDUCE);
    launch_reduce_parts(s.d_part.as<z64>(), s.nsplit, n, s.nv, nullptr, -1.0, s.d_C.as<z64>(),
                        st_);
    prof_end(h, (s.nsplit + 1.0) * n * s.nv * sizeof(z64), 0.0);
    h = prof_begin(PH_GEMM_AC);
    launch_gemm_a_c(s.W(), s.npw, s.nv, s.d_C.as<z64>(), v, dl, n, s.npw, 1.0, dot_in, dd, st_);
    prof_end(h, s.nv * vb + n * vb * (dots ? 3.0 : 2.0), gf);
  } else {
    z32* part = reinterpret_cast<z32*>(s.d_part.as<z64>());
    z32* C = reinterpret_cast<z32*>(s.d_C.as<z64>());
    launch_gemm_ah_b(s.d_W32.as<z32>(), s.npw, s.nv, {v.base, v.stride}, dl, n, s.npw, s.kchunk,
                     part, st_);
    prof_end(h, s.nv * vb / 2 + n * vb, gf);
    h = prof_begin(PH_REDUCE);
    launch_reduce_parts(part, s.nsplit, n, s.nv, nullptr, -1.0, C, st_);
    prof_end(h, (s.nsplit + 1.0) * n * s.nv * sizeof(z32), 0.0);
    h = prof_begin(PH_GEMM_AC);
    launch_gemm_a_c(s.d_W32.as<z32>(), s.npw, s.nv, C, v, dl, n, s.npw, 1.0, dot_in, dd, st_);
    prof_end(h, s.nv * vb / 2 + n * vb * (dots ? 3.0 : 2.0), gf);
  }
}

// ------------------------------------------------------------------ profiling
void Context::profile(bool on) {
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  prof_harvest();
  prof_on_ = on;
}

int Context::prof_begin(int phase) {
  if (!prof_on_) return -1;
  std::lock_guard<std::mutex> lk(prof_mu_);
  ProfRec r{phase, nullptr, nullptr, 0.0, 0.0};
  for (hipEvent_t* e : {&r.a, &r.b}) {
    if (!ev_pool_.empty()) {
      *e = ev_pool_.back();
      ev_pool_.pop_back();
    } else {
      STH_HIP_CHECK(hipEventCreate(e));
    }
  }
  STH_HIP_CHECK(hipEventRecord(r.a, st_));
  prof_recs_.push_back(r);
  return int(prof_recs_.size()) - 1;
}

void Context::prof_end(int handle, double bytes, double flops) {
  if (handle < 0) return;
  std::lock_guard<std::mutex> lk(prof_mu_);
  ProfRec& r = prof_recs_[handle];
  r.bytes = bytes;
  r.flops = flops;
  STH_HIP_CHECK(hipEventRecord(r.b, st_));
}

void Context::prof_harvest() {
  std::lock_guard<std::mutex> lk(prof_mu_);
  for (ProfRec& r : prof_recs_) {
    float ms = 0.0f;
    STH_HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
    prof_ms_[r.phase] += ms;
    prof_bytes_[r.phase] += r.bytes;
    prof_flops_[r.phase] += r.flops;
    prof_n_[r.phase] += 1;
    ev_pool_.push_back(r.a);
    ev_pool_.push_back(r.b);
  }
  prof_recs_.clear();
}

void Context::profile_read(double* ms, long long* n, double* bytes, double* flops) {
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  prof_harvest();
  std::lock_guard<std::mutex> lk(prof_mu_);
  for (int p = 0; p < NPH; ++p) {
    if (ms) ms[p] = prof_ms_[p];
    if (n) n[p] = prof_n_[p];
    if (bytes) bytes[p] = prof_bytes_[p];
    if (flops) flops[p] = prof_flops_[p];
    prof_ms_[p] = prof_bytes_[p] = prof_flops_[p] = 0.0;
    prof_n_[p] = 0;
  }
}

void Context::h_scratch(System& s, HScratch& w, int cap) {
  const int mp = std::max(s.nproj, 1);
  w.cap = cap;
  w.sticks = DevMem(&budget_, (size_t)cap * s.N * s.nst * sizeof(z64));
  w.part = DevMem(&budget_, (size_t)s.nsplit * cap * mp * sizeof(z64));
  w.C = DevMem(&budget_, (size_t)cap * mp * sizeof(z64));
  w.zeros = DevMem(&budget_, (size_t)cap * sizeof(double));
  w.ids = DevMem(&budget_, (size_t)cap * sizeof(int));
  w.zeros.zero(st_);
  std::vector<int> idv(cap);
  std::iota(idv.begin(), idv.end(), 0);
  STH_HIP_CHECK(hipMemcpyAsync(w.ids.as<void>(), idv.data(), cap * sizeof(int),
                               hipMemcpyHostToDevice, st_));
  STH_HIP_CHECK(hipStreamSynchronize(st_));
}

// out = H in for n contiguous vectors (internal order): T + V_loc by the
// dual-space FFT route, V_NL by the projector GEMMs.
void Context::h_block(System& s, HScratch& w, const z64* in, z64* out, int n) {
  HView v;
  v.sticks = w.sticks.as<z64>();
  v.part = w.part.as<z64>();
  v.C = w.C.as<z64>();
  v.zeros = w.zeros.as<double>();
  v.ids = w.ids.as<int>();
  v.cap = w.cap;
  h_block_on(s, v, in, out, n, st_);
}

void Context::h_block_on(System& s, const HView& w, const z64* in, z64* out, int n,
                         hipStream_t st_) {
  const int N = s.N;
  for (int c0 = 0; c0 < n; c0 += w.cap) {
    const int nc = std::min(w.cap, n - c0);
    VecSet<const z64> vin{in + (size_t)c0 * s.npw, (long long)s.npw};
    VecSet<z64> vout{out + (size_t)c0 * s.npw, (long long)s.npw};
    VecSet<z64> st{w.sticks, (long long)N * s.nst};
    const int* ids = w.ids;
    launch_zfft_inv<double, z64>(s.g, vin, st, ids, nc, st_);
    launch_plane_local<double>(s.g, st, ids, nc, s.d_vloc.as<double>(), nullptr, st_);
    launch_zfft_fwd<double, z64>(s.g, {st.base, st.stride}, vout, ids, nc, ZF_SHIFT, vin, w.zeros,
                                 st_);
    if (s.nproj) {
      launch_gemm_ah_b(s.beta(), s.npw, s.nproj, vin, ids, nc, s.npw, s.kchunk, w.part, st_);
      launch_reduce_parts(w.part, s.nsplit, nc, s.nproj, s.d_diag.as<double>() + s.nv, 1.0, w.C,
                          st_);
      launch_gemm_a_c(s.beta(), s.npw, s.nproj, w.C, vout, ids, nc, s.npw, 1.0, {nullptr, 0},
                      nullptr, st_);
    }
  }
}

void Context::apply_h(int id, int nvec, const double* in, double* out, int ptr_kind,
                      hipStream_t user) {
  check_ptr_kind(ptr_kind);
  if (nvec < 0 || (nvec > 0 && (!in || !out))) {
    set_error("apply_h: nvec >= 0 and non-null in/out required");
    throw Error(STH_E_INVALID);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System& s = sys(id);
  if (nvec == 0) return;
  order_after(user);
  const int chunk = std::min(nvec, 256);
  const size_t vb = (size_t)s.npw * sizeof(z64);
  DevMem tin(&budget_, (size_t)chunk * vb), tout(&budget_, (size_t)chunk * vb);
  DevMem a(&budget_, (size_t)chunk * vb), bq(&budget_, (size_t)chunk * vb);
  HScratch w;
  h_scratch(s, w, chunk);
  for (int c0 = 0; c0 < nvec; c0 += chunk) {
    const int nc = std::min(chunk, nvec - c0);
    copy_in(tin.as<void>(), in + (size_t)c0 * s.npw * 2, (size_t)nc * vb, ptr_kind, st_);
    launch_permute_in(tin.as<z64>(), s.npw, a.as<z64>(), s.npw, s.d_perm.as<int>(), s.npw, nc,
                      st_);
    h_block(s, w, a.as<z64>(), bq.as<z64>(), nc);
    launch_permute_out(bq.as<z64>(), s.npw, tout.as<z64>(), s.npw, s.d_perm.as<int>(), s.npw, nc,
                       st_);
    copy_out(out + (size_t)c0 * s.npw * 2, tout.as<void>(), (size_t)nc * vb, ptr_kind, st_);
  }
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  order_before(user);
}

// ------------------------------------------------------------------ requests
uint64_t Context::submit(int id, int npert, const double* dv, int nband, const int32_t* bands,
                         const sth_solve_opts& o, int ptr_kind, hipStream_t user) {
  check_ptr_kind(ptr_kind);
  if (npert <= 0 || nband <= 0 || !dv || !bands) {
    set_error("submit: npert > 0, nband > 0, dv_r and bands required");
    throw Error(STH_E_INVALID);
  }
  if (!(o.tol > 0.0) || o.maxit < 0 ||
      (o.precision != STH_FP64 && o.precision != STH_MIXED && o.precision != STH_MIXED_BF16)) {
    set_error("submit: tol > 0, maxit >= 0 and precision STH_FP64 / STH_MIXED / "
              "STH_MIXED_BF16 required");
    throw Error(STH_E_INVALID);
  }
  auto queued = [&]() {   // requests waiting for admission, all systems (mu_ held)
    size_t q = 0;
    for (auto& kv : systems_) q += kv.second->waiting.size();
    return q;
  };
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (queued() >= size_t(max_queued_)) {
      set_error("submit: %d requests are already waiting for admission", max_queued_);
      throw Error(STH_E_AGAIN);
    }
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System& s = sys(id);
  std::set<int> seen;
  for (int i = 0; i < nband; ++i) {
    if (bands[i] < 0 || bands[i] >= s.nv || !seen.insert(bands[i]).second) {
      set_error("submit: band %d out of range [0, %d) or repeated", bands[i], s.nv);
      throw Error(STH_E_INVALID);
    }
  }
  const long long n3 = (long long)s.N * s.N * s.N;
  // smallest footprint the request can run in: dV and Delta n, and the Delta psi
  // of every perturbation (want_dpsi) or of one perturbation at a time; it must
  // fit the budget left by the resident systems (requests and tickets come and go)
  const size_t need = (size_t)npert * n3 * 8 * 2 +
                      (size_t)(o.want_dpsi ? npert : 1) * nband * s.npw * 16 + nband * 4;
  size_t resident = 0;
  for (auto& kv : systems_) resident += kv.second->resident_bytes;
  const size_t room = budget_.limit() - std::min(budget_.limit(), resident);
  if (need > room) {
    set_error("request needs %zu bytes, more than the %zu the budget leaves next to the "
              "resident systems", need, room);
    throw Error(STH_E_NOMEM);
  }
  auto r = std::make_shared<Request>();
  r->sys_id = id;
  r->sys = &s;
  r->npert = npert;
  r->nband = nband;
  r->bands.assign(bands, bands + nband);
  r->tol = o.tol;
  r->maxit = o.maxit > 0 ? o.maxit : 1000;
  r->precision = o.precision;
  r->want_dpsi = o.want_dpsi;
  r->d_dv = DevMem(&budget_, (size_t)npert * n3 * sizeof(double));
  order_after(user);
  copy_in(r->d_dv.as<void>(), dv, (size_t)npert * n3 * sizeof(double), ptr_kind, st_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  const int ns = npert * nband;
  r->iters.assign(ns, 0);
  r->status.assign(ns, -1);
  r->resid.assign(ns, 0.0);
  r->latency.assign(ns, 0.0);
  r->pert_left.assign(npert, nband);
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(mu_);
  if (queued() >= size_t(max_queued_)) {   // filled by another thread meanwhile
    set_error("submit: %d requests are already waiting for admission", max_queued_);
    throw Error(STH_E_AGAIN);
  }
  r->ticket = next_ticket_++;
  tickets_[r->ticket] = r;
  s.waiting.push_back(r);
  ++mem_epoch_;
  cv_.notify_all();
  return r->ticket;
}

void Context::poll(uint64_t t, sth_ticket_info* info) {
  auto r = find(t);
  std::lock_guard<std::mutex> lk(mu_);
  if (r->failed) {
    set_error("ticket %llu failed", (unsigned long long)t);
    throw Error(r->fail_code ? r->fail_code : STH_E_INTERNAL);
  }
  info->state = r->state;
  info->n_total = r->npert * r->nband;
  info->n_finished = r->n_finished;
  info->n_converged = r->n_converged;
  info->max_rel_resid = r->max_resid;
  info->t_submit = r->t_submit;
  info->t_start = r->t_start;
  info->t_done = r->t_done;
  info->cg_iterations = r->cg_its;
  info->op_applications = r->op_apps;
  info->op_applications_fp32 = r->op32_apps;
  const auto sit = systems_.find(r->sys_id);   // the system may have been released
  info->graph_replays = sit != systems_.end() ? sit->second->graph_replays : 0;
  info->system_id = r->sys_id;
  info->npert = r->npert;
  info->nband = r->nband;
}

bool Context::wait(uint64_t t, double timeout) {
  auto r = find(t);
  std::unique_lock<std::mutex> lk(mu_);
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(timeout, 0.0));
  while (r->state < 2) {
    if (cv_.wait_until(lk, deadline) == std::cv_status::timeout && r->state < 2) return false;
  }
  if (r->failed) {
    set_error("ticket %llu failed", (unsigned long long)t);
    throw Error(r->fail_code ? r->fail_code : STH_E_INTERNAL);
  }
  return true;
}

static void require_done(const Request& r) {
  if (r.failed) {
    set_error("ticket failed");
    throw Error(r.fail_code ? r.fail_code : STH_E_INTERNAL);
  }
  if (r.state != 2) {
    set_error("ticket not finished");
    throw Error(STH_E_NOT_READY);
  }
}

void Context::fetch_drho(uint64_t t, double* out, int ptr_kind, hipStream_t user) {
  check_ptr_kind(ptr_kind);
  auto r = find(t);
  {
    std::lock_guard<std::mutex> lk(mu_);
    require_done(*r);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  order_after(user);
  copy_out(out, r->d_drho.as<void>(), r->d_drho.bytes(), ptr_kind, st_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  order_before(user);
}

void Context::fetch_dpsi(uint64_t t, double* out, int ptr_kind, hipStream_t user) {
  check_ptr_kind(ptr_kind);
  auto r = find(t);
  {
    std::lock_guard<std::mutex> lk(mu_);
    require_done(*r);
  }
  if (!r->want_dpsi) {
    set_error("fetch_dpsi: the request was submitted without want_dpsi");
    throw Error(STH_E_INVALID);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System& s = sys(r->sys_id);
  order_after(user);
  for (int j = 0; j < r->npert; ++j)
    if (r->blk_of[j] != j) {   // want_dpsi requests keep block j for perturbation j
      set_error("fetch_dpsi: Delta psi block of perturbation %d missing", j);
      throw Error(STH_E_INTERNAL);
    }
  const int nv = r->npert * r->nband;
  const int chunk = std::min(nv, 1024);
  DevMem tmp(&budget_, (size_t)chunk * s.npw * sizeof(z64));
  for (int c0 = 0; c0 < nv; c0 += chunk) {
    const int nc = std::min(chunk, nv - c0);
    launch_permute_out(r->d_dpsi.as<z64>() + (size_t)c0 * s.npw, s.npw, tmp.as<z64>(), s.npw,
                       s.d_perm.as<int>(), s.npw, nc, st_);
    copy_out(out + (size_t)c0 * s.npw * 2, tmp.as<void>(), (size_t)nc * s.npw * sizeof(z64),
             ptr_kind, st_);
  }
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  order_before(user);
}

void Context::fetch_stats(uint64_t t, int32_t* iters, double* resid, int32_t* status,
                          double* lat) {
  auto r = find(t);
  std::lock_guard<std::mutex> lk(mu_);
  require_done(*r);
  const int n = r->npert * r->nband;
  for (int i = 0; i < n; ++i) {
    if (iters) iters[i] = r->iters[i];
    if (resid) resid[i] = r->resid[i];
    if (status) status[i] = r->status[i];
    if (lat) lat[i] = r->latency[i];
  }
}

void Context::release_ticket(uint64_t t) {
  std::lock_guard<std::mutex> glk(gpu_mu_);
  std::lock_guard<std::mutex> lk(mu_);
  auto it = tickets_.find(t);
  if (it == tickets_.end()) {
    set_error("unknown ticket %llu", (unsigned long long)t);
    throw Error(STH_E_NOT_FOUND);
  }
  if (it->second->state == 1) {
    set_error("ticket %llu is running", (unsigned long long)t);
    throw Error(STH_E_NOT_READY);
  }
  if (it->second->state == 0) {   // still waiting: withdraw it
    for (auto& kv : systems_) {
      auto& w = kv.second->waiting;
      w.erase(std::remove(w.begin(), w.end(), it->second), w.end());
    }
  }
  tickets_.erase(it);
  ++mem_epoch_;
  cv_.notify_all();
}

// ------------------------------------------------------------------ server
void Context::server_loop() {
  (void)hipSetDevice(device_);
  while (true) {
    std::vector<System*> work;
    {
      std::unique_lock<std::mutex> lk(mu_);
      // a system has work when it runs requests, or holds waiting ones and memory
      // may have been freed since admission last found no room
      auto busy = [&](const System& sy) {
        return !sy.running.empty() || (!sy.waiting.empty() && sy.blocked_epoch != mem_epoch_);
      };
      cv_.wait(lk, [&] {
        if (stop_) return true;
        for (auto& kv : systems_)
          if (busy(*kv.second)) return true;
        return false;
      });
      if (stop_) return;
      for (auto& kv : systems_)
        if (busy(*kv.second)) work.push_back(kv.second.get());
    }
    for (System* sp : work) {
      std::lock_guard<std::mutex> glk(gpu_mu_);
      {
        std::lock_guard<std::mutex> lk(mu_);
        bool alive = false;
        for (auto& kv : systems_) alive |= (kv.second.get() == sp);
        if (!alive) continue;
      }
      try {
        step(*sp);
      } catch (const Error& e) {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& r : sp->running) {
          r->failed = true;
          r->fail_code = e.code;
          r->state = 3;
        }
        sp->running.clear();
        for (auto& sl : sp->slots) sl = SlotHost{};
        cv_.notify_all();
      }
    }
  }
}

void Context::admit(System& s) {
  std::lock_guard<std::mutex> lk(mu_);
  while (!s.waiting.empty()) {
    auto r = s.waiting.front();
    const long long n3 = (long long)s.N * s.N * s.N;
    const size_t blk = (size_t)r->nband * s.npw * sizeof(z64);
    const size_t fixed = (size_t)r->npert * n3 * sizeof(double) + r->nband * sizeof(int);
    // Delta psi window: every perturbation when the caller fetches Delta psi;
    // otherwise enough perturbations to fill every slot plus one whose Delta n
    // is being formed, fewer if the budget is short (down to one)
    const int lo = r->want_dpsi ? r->npert : 1;
    int win = r->want_dpsi ? r->npert
                           : std::min(r->npert, (s.nslots + r->nband - 1) / r->nband + 1);
    while (win > lo && !budget_.fits(fixed + win * blk)) --win;
    const size_t need = fixed + win * blk;
    if (!budget_.fits(need)) {
      // it fits once requests finish and their tickets are released (submit
      // checked the room next to the resident systems); until then it waits,
      // and with nothing of this system running the server sleeps until memory
      // may have been freed
      if (s.running.empty()) s.blocked_epoch = mem_epoch_;
      break;
    }
    r->d_dpsi = DevMem(&budget_, win * blk);
    r->win = win;
    r->blk_of.assign(r->npert, -1);
    r->free_blk.clear();
    for (int b = 0; b < win; ++b) r->free_blk.push_back(b);
    r->d_drho = DevMem(&budget_, (size_t)r->npert * n3 * sizeof(double));
    r->d_bands = DevMem(&budget_, (size_t)r->nband * sizeof(int));
    STH_HIP_CHECK(hipMemcpyAsync(r->d_bands.as<void>(), r->bands.data(), r->nband * sizeof(int),
                                 hipMemcpyHostToDevice, st_));
    r->state = 1;
    r->t_start = now_s();
    s.running.push_back(r);
    s.waiting.pop_front();
  }
}

void Context::refill(System& s) {
  std::vector<int> fresh, band;
  double* h_eps = s.h_eps.as<double>();
  double* h_ekin = h_eps + s.nslots;
  double* h_tol = h_eps + 2 * s.nslots;
  int* h_maxit = reinterpret_cast<int*>(h_eps + 3 * s.nslots);
  int* h_prec = reinterpret_cast<int*>(h_eps + 4 * s.nslots);
  const double** h_pp = s.h_potptr.as<const double*>();
  const long long n3 = (long long)s.N * s.N * s.N;
  const double t = now_s();
  int slot = 0;
  for (auto& r : s.running) {
    const int total = r->npert * r->nband;
    while (r->next < total) {
      while (slot < s.nslots && s.slots[slot].req) ++slot;
      if (slot >= s.nslots) break;
      // a perturbation starts only with a Delta psi block of its own
      const int jn = r->next / r->nband;
      if (r->blk_of[jn] < 0) {
        if (r->free_blk.empty()) break;
        r->blk_of[jn] = r->free_blk.front();
        r->free_blk.pop_front();
      }
      const int solve = r->next++;
      const int j = solve / r->nband, vi = solve % r->nband, v = r->bands[vi];
      s.slots[slot] = SlotHost{r.get(), solve, t, 0};
      h_eps[slot] = s.eps[v];
      h_ekin[slot] = s.ekin[v];
      h_tol[slot] = r->tol;
      h_maxit[slot] = r->maxit;
      h_prec[slot] = r->precision != STH_FP64 ? 1 : 0;
      h_pp[slot] = r->d_dv.as<double>() + j * n3;
      fresh.push_back(slot);
      band.push_back(v);
    }
    if (slot >= s.nslots) break;
  }
  if (fresh.empty()) return;
  const int n = int(fresh.size());
  // per-slot constants: eps, ekin, tol (doubles) and maxit (ints)
  STH_HIP_CHECK(hipMemcpyAsync(s.ss.eps, h_eps, s.nslots * sizeof(double), hipMemcpyHostToDevice,
                               st_));
  STH_HIP_CHECK(hipMemcpyAsync(s.ss.ekin, h_ekin, s.nslots * sizeof(double),
                               hipMemcpyHostToDevice, st_));
  STH_HIP_CHECK(hipMemcpyAsync(s.ss.tol, h_tol, s.nslots * sizeof(double), hipMemcpyHostToDevice,
                               st_));
  STH_HIP_CHECK(hipMemcpyAsync(s.ss.maxit, h_maxit, s.nslots * sizeof(int), hipMemcpyHostToDevice,
                               st_));
  STH_HIP_CHECK(hipMemcpyAsync(s.ss.prec, h_prec, s.nslots * sizeof(int), hipMemcpyHostToDevice,
                               st_));
  STH_HIP_CHECK(hipMemcpyAsync(s.d_potptr.as<void>(), h_pp, s.nslots * sizeof(double*),
                               hipMemcpyHostToDevice, st_));
  int* dl = upload_list(s, fresh);
  int* db = upload_list(s, band);
  const int N = s.N;
  VecSet<z64> sticks{s.d_sticks.as<z64>(), (long long)N * s.nst};
  // u = FFT[dV_j(r) psi_v(r)] on the sphere, then b = -P_c u = Psi (Psi^H u) - u
  const int hrhs = prof_begin(PH_OTHER);
  launch_copy_vecs({s.W(), (long long)s.npw}, s.vec(s.d_p), db, dl, n, s.npw, st_);
  launch_zfft_inv<double, z64>(s.g, s.cvec(s.d_p), sticks, dl, n, st_);
  launch_plane_local<double>(s.g, sticks, dl, n, nullptr, s.d_potptr.as<const double* const>(),
                             st_);
  launch_zfft_fwd<double, z64>(s.g, {sticks.base, sticks.stride}, s.vec(s.d_b), dl, n, ZF_PLAIN,
                               {nullptr, 0}, nullptr, st_);
  if (s.gamma) {
    gamma_pair<double>(s, s.W(), s.nv, nullptr, 1.0, s.cvec(s.d_b), s.vec(s.d_b), dl, n, -1.0,
                       {nullptr, 0}, nullptr, s.d_part.as<z64>(), s.d_C.as<z64>(), false);
  } else {
  launch_gemm_ah_b(s.W(), s.npw, s.nv, s.cvec(s.d_b), dl, n, s.npw, s.kchunk, s.d_part.as<z64>(),
                   st_);
  launch_reduce_parts(s.d_part.as<z64>(), s.nsplit, n, s.nv, nullptr, 1.0, s.d_C.as<z64>(), st_);
  launch_gemm_a_c(s.W(), s.npw, s.nv, s.d_C.as<z64>(), s.vec(s.d_b), dl, n, s.npw, -1.0,
                  {nullptr, 0}, nullptr, st_);
  }
  launch_cg_init(s.g, s.cvec(s.d_b), s.vec(s.d_x), s.vec(s.d_r), s.vec(s.d_p), dl, n, s.ss.ekin,
                 s.d_part2.as<double>(), st_);
  launch_cg_init_scalars(s.d_part2.as<double>(), s.nchunk, dl, n, s.ss, st_);
  prof_end(hrhs, 0.0, 0.0);
}

// One CG iteration on the listed slots: q = A p (FP64 or FP32 operator) with
// <p, q> partials, alpha, x/r update with <r, K r> and ||r||^2, beta and the
// convergence test, p = K r + beta p.
void Context::cg_step(System& s, const int* dl, int n, int mode) {
  const double vb = double(s.npw) * sizeof(z64);
  apply_op(s, s.cvec(s.d_p), s.vec(s.d_q), dl, n, false, mode);
  project_c(s, s.vec(s.d_q), dl, n, s.cvec(s.d_p), true, mode);
  const int h = prof_begin(PH_CG);
  launch_cg_alpha(s.d_dots.as<double>(), s.ntile, dl, n, s.ss, st_);
  launch_cg_update_xr(s.g, s.vec(s.d_x), s.vec(s.d_r), s.cvec(s.d_p), s.cvec(s.d_q), dl, n, s.ss,
                      s.d_part2.as<double>(), st_);
  launch_cg_beta(s.d_part2.as<double>(), s.nchunk, dl, n, s.ss, st_);
  launch_cg_update_p(s.g, s.cvec(s.d_r), s.vec(s.d_p), dl, n, s.ss, st_);
  prof_end(h, n * 9.0 * vb + 2.0 * s.npw * 8.0, 0.0);
}

void Context::iterate(System& s, const std::vector<int>& act, int nit) {
  // slots grouped by operator form (FP64, FP32 inner operator with FP32 or BF16
  // projector GEMMs) iterate as separate batches; partial sums are indexed by
  // list position, so each batch runs its whole CG step before the next starts
  std::vector<int> lists[3];
  for (int slot : act) lists[s.slots[slot].req->precision].push_back(slot);
  // steady state: every slot holds a solve of one form -> replay the captured
  // graph of nit iterations over the identity list (kernels skip slots that are
  // no longer ACTIVE).  The per-kernel profiler needs direct launches.
  int kall = -1;
  for (int k = 0; k < 3; ++k)
    if (int(lists[k].size()) == int(act.size())) kall = k;
  if (use_graphs_ && !prof_on_ && kall >= 0 && int(act.size()) == s.nslots) {
    if (!s.graph[kall] || s.graph_nit[kall] != nit) {
      if (s.graph[kall]) STH_HIP_CHECK(hipGraphExecDestroy(s.graph[kall]));
      s.graph[kall] = nullptr;
      hipGraph_t gr = nullptr;
      STH_HIP_CHECK(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      for (int it = 0; it < nit; ++it) cg_step(s, s.d_ident.as<int>(), s.nslots, kall);
      STH_HIP_CHECK(hipStreamEndCapture(st_, &gr));
      STH_HIP_CHECK(hipGraphInstantiate(&s.graph[kall], gr, nullptr, nullptr, 0));
      STH_HIP_CHECK(hipGraphDestroy(gr));
      s.graph_nit[kall] = nit;
    }
    STH_HIP_CHECK(hipGraphLaunch(s.graph[kall], st_));
    s.graph_replays += 1;
  } else {
    int* dl[3] = {nullptr, nullptr, nullptr};
    for (int k = 0; k < 3; ++k)
      if (!lists[k].empty()) dl[k] = upload_list(s, lists[k]);
    for (int it = 0; it < nit; ++it)
      for (int k = 0; k < 3; ++k)
        if (!lists[k].empty()) cg_step(s, dl[k], int(lists[k].size()), k);
  }
  std::lock_guard<std::mutex> lk(mu_);
  for (int slot : act) {
    s.slots[slot].req->op_apps += nit;
    if (s.slots[slot].req->precision != STH_FP64) s.slots[slot].req->op32_apps += nit;
  }
}

void Context::check_and_retire(System& s, std::vector<int>& act) {
  int* h_status = s.h_status.as<int>();
  int* h_iters = h_status + s.nslots;
  double* h_rn2 = s.h_rn2.as<double>();
  double* h_bn2 = h_rn2 + s.nslots;
  auto read_state = [&]() {
    STH_HIP_CHECK(hipMemcpyAsync(h_status, s.ss.status, s.nslots * sizeof(int),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipMemcpyAsync(h_iters, s.ss.iters, s.nslots * sizeof(int),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipMemcpyAsync(h_rn2, s.ss.rnorm2, s.nslots * sizeof(double),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipMemcpyAsync(h_bn2, s.ss.bnorm2, s.nslots * sizeof(double),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
  };
  read_state();
  std::vector<int> check;
  for (int i = 0; i < s.nslots; ++i)
    if (s.slots[i].req && h_status[i] == SLOT_CHECK) check.push_back(i);
  if (!check.empty()) {
    const int n = int(check.size());
    // true residual r = P_c (b - (H - eps) P_c x) of the candidates.  x is
    // projected first: the P_v parts of the directions it accumulated meet
    // (H - eps) Psi = Psi (Lambda - eps) only as far as the valence states
    // are eigenvectors, so they could bias the check
    int* dl = upload_list(s, check);
    project_c(s, s.vec(s.d_x), dl, n, {nullptr, 0}, false, OP_FP64);
    apply_op(s, s.cvec(s.d_x), s.vec(s.d_q), dl, n, false);
    project_c(s, s.vec(s.d_q), dl, n, {nullptr, 0}, false, OP_FP64);
    launch_cg_true_resid(s.g, s.cvec(s.d_b), s.cvec(s.d_q), s.vec(s.d_r), dl, n, s.ss.ekin,
                         s.d_part2.as<double>(), st_);
    launch_cg_check_true(s.d_part2.as<double>(), s.nchunk, dl, n, s.ss, st_);
    launch_cg_update_p(s.g, s.cvec(s.d_r), s.vec(s.d_p), dl, n, s.ss, st_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (int slot : check) s.slots[slot].req->op_apps += 1;
    }
    read_state();
  }
  // solves that stopped inside the recurrence (maxit in the beta step, breakdown)
  // report the true FP64 residual of their last iterate, not the recursive one
  // (for mixed solves that would be the residual of the inner operator)
  std::vector<int> stopped;
  for (int i = 0; i < s.nslots; ++i)
    if (s.slots[i].req && (h_status[i] == SLOT_MAXIT || h_status[i] == SLOT_BREAKDOWN))
      stopped.push_back(i);
  if (!stopped.empty()) {
    const int n = int(stopped.size());
    int* dl = upload_list(s, stopped);
    project_c(s, s.vec(s.d_x), dl, n, {nullptr, 0}, false, OP_FP64);
    apply_op(s, s.cvec(s.d_x), s.vec(s.d_q), dl, n, false);
    project_c(s, s.vec(s.d_q), dl, n, {nullptr, 0}, false, OP_FP64);
    launch_cg_true_resid(s.g, s.cvec(s.d_b), s.cvec(s.d_q), s.vec(s.d_r), dl, n, s.ss.ekin,
                         s.d_part2.as<double>(), st_);
    launch_cg_check_true(s.d_part2.as<double>(), s.nchunk, dl, n, s.ss, st_, true);
    read_state();
  }
  std::vector<int> fin;
  for (int i = 0; i < s.nslots; ++i)
    if (s.slots[i].req && h_status[i] >= SLOT_DONE) fin.push_back(i);
  if (fin.empty()) return;
  const int n = int(fin.size());
  int* dl = upload_list(s, fin);
  // x <- P_c x, then store into the owning request's dpsi
  if (s.gamma) {
    gamma_pair<double>(s, s.W(), s.nv, nullptr, -1.0, s.cvec(s.d_x), s.vec(s.d_x), dl, n, 1.0,
                       {nullptr, 0}, nullptr, s.d_part.as<z64>(), s.d_C.as<z64>(), false);
  } else {
  launch_gemm_ah_b(s.W(), s.npw, s.nv, s.cvec(s.d_x), dl, n, s.npw, s.kchunk, s.d_part.as<z64>(),
                   st_);
  launch_reduce_parts(s.d_part.as<z64>(), s.nsplit, n, s.nv, nullptr, -1.0, s.d_C.as<z64>(), st_);
  launch_gemm_a_c(s.W(), s.npw, s.nv, s.d_C.as<z64>(), s.vec(s.d_x), dl, n, s.npw, 1.0,
                  {nullptr, 0}, nullptr, st_);
  }
  std::map<Request*, std::pair<std::vector<int>, std::vector<int>>> by_req;
  for (int slot : fin) {
    Request* r = s.slots[slot].req;
    const int solve = s.slots[slot].solve;
    auto& e = by_req[r];
    e.first.push_back(slot);
    e.second.push_back(r->blk_of[solve / r->nband] * r->nband + solve % r->nband);
  }
  for (auto& kv : by_req) {
    int* ds = upload_list(s, kv.second.first);
    int* dd = upload_list(s, kv.second.second);
    launch_copy_vecs(s.cvec(s.d_x), {kv.first->d_dpsi.as<z64>(), (long long)s.npw}, ds, dd,
                     int(kv.second.first.size()), s.npw, st_);
  }
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  const double t = now_s();
  std::lock_guard<std::mutex> lk(mu_);
  for (int slot : fin) {
    SlotHost& sh = s.slots[slot];
    Request* r = sh.req;
    const int st = h_status[slot];
    const double rel = h_bn2[slot] > 0 ? std::sqrt(h_rn2[slot] / h_bn2[slot]) : 0.0;
    r->iters[sh.solve] = h_iters[slot];
    r->resid[sh.solve] = rel;
    r->status[sh.solve] = st == SLOT_DONE        ? STH_SOLVE_CONVERGED
                          : st == SLOT_MAXIT     ? STH_SOLVE_MAXIT
                          : st == SLOT_BREAKDOWN ? STH_SOLVE_BREAKDOWN
                                                 : STH_SOLVE_NAN;
    r->latency[sh.solve] = t - sh.t_admit;
    r->cg_its += h_iters[slot];
    r->n_finished += 1;
    if (st == SLOT_DONE) r->n_converged += 1;
    if (rel > r->max_resid || rel != rel) r->max_resid = rel;
    const int j = sh.solve / r->nband;
    if (--r->pert_left[j] == 0) r->drho_pending.push_back(j);
    sh = SlotHost{};
  }
  act.clear();
}

void Context::finish_drho(System& s) {
  const long long n3 = (long long)s.N * s.N * s.N;
  std::vector<std::shared_ptr<Request>> run;
  {
    std::lock_guard<std::mutex> lk(mu_);
    run = s.running;
  }
  for (auto& r : run) {
    std::vector<int> todo;
    {
      std::lock_guard<std::mutex> lk(mu_);
      todo.swap(r->drho_pending);
    }
    for (int j : todo) {
      std::vector<int> id(r->nband);
      std::iota(id.begin(), id.end(), 0);
      int* dl = upload_list(s, id);
      VecSet<z64> sticks{s.d_drho_sticks.as<z64>(), (long long)s.N * s.nst};
      launch_zfft_inv<double, z64>(
          s.g,
          {r->d_dpsi.as<const z64>() + (size_t)r->blk_of[j] * r->nband * s.npw, (long long)s.npw},
          sticks, dl, r->nband, st_);
      launch_drho(s.g, s.d_drho_sticks.as<z64>(), (long long)s.N * s.nst, r->nband,
                  r->d_bands.as<int>(), s.d_psir.as<z64>(), 1, 2.0 * s.fs / s.omega,
                  r->d_drho.as<double>() + j * n3, st_);
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      s.lists_used -= r->nband;
      std::lock_guard<std::mutex> lk(mu_);
      r->n_drho_done += 1;
      if (!r->want_dpsi) {   // the block serves the next perturbation
        r->free_blk.push_back(r->blk_of[j]);
        r->blk_of[j] = -1;
      }
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (r->n_finished == r->npert * r->nband && r->n_drho_done == r->npert) {
      r->state = 2;
      r->t_done = now_s();
      s.running.erase(std::remove(s.running.begin(), s.running.end(), r), s.running.end());
      cv_.notify_all();
    }
  }
}

bool Context::step(System& s) {
  STH_HIP_CHECK(hipSetDevice(device_));
  s.lists_used = 0;
  admit(s);
  refill(s);
  std::vector<int> act;
  for (int i = 0; i < s.nslots; ++i)
    if (s.slots[i].req) act.push_back(i);
  if (!act.empty()) {
    iterate(s, act, check_every_);
    check_and_retire(s, act);
  }
  finish_drho(s);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  prof_harvest();
  return true;
}

void Context::chi0_block(uint64_t t, double* M, double* S, double* lam) {
  auto r = find(t);
  {
    std::lock_guard<std::mutex> lk(mu_);
    require_done(*r);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System& s = sys(r->sys_id);
  const int np = r->npert;
  const long long n3 = (long long)s.N * s.N * s.N;
  const int K = int(n3 / 2);   // a real n^3 vector read as n^3/2 complex numbers
  const double w = s.omega / double(n3);
  const int kchunk = 16384;
  const int nsplit = (K + kchunk - 1) / kchunk;
  DevMem part(&budget_, (size_t)nsplit * np * np * sizeof(z64));
  DevMem C(&budget_, (size_t)np * np * sizeof(z64));
  DevMem ids(&budget_, (size_t)np * sizeof(int));
  std::vector<int> idv(np);
  std::iota(idv.begin(), idv.end(), 0);
  STH_HIP_CHECK(
      hipMemcpyAsync(ids.as<void>(), idv.data(), np * sizeof(int), hipMemcpyHostToDevice, st_));
  std::vector<z64> hc((size_t)np * np);
  std::vector<double> Mh((size_t)np * np), Sh((size_t)np * np);
  for (int pass = 0; pass < 2; ++pass) {
    // Re(sum_k conj(a_k) b_k) over complex pairs = real dot product over n^3
    const z64* A = r->d_dv.as<const z64>();
    const z64* B = pass == 0 ? r->d_drho.as<const z64>() : r->d_dv.as<const z64>();
    launch_gemm_ah_b(A, K, np, {B, K}, ids.as<int>(), np, K, kchunk, part.as<z64>(), st_);
    launch_reduce_parts(part.as<z64>(), nsplit, np, np, nullptr, w, C.as<z64>(), st_);
    STH_HIP_CHECK(hipMemcpyAsync(hc.data(), C.as<void>(), hc.size() * sizeof(z64),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    // C[c][m] = sum conj(A_m) B_c: row i = m (dV_i), column j = c
    std::vector<double>& out = pass == 0 ? Mh : Sh;
    for (int j = 0; j < np; ++j)
      for (int i = 0; i < np; ++i) out[(size_t)i * np + j] = hc[(size_t)j * np + i].x;
  }
  if (M) std::memcpy(M, Mh.data(), Mh.size() * sizeof(double));
  if (S) std::memcpy(S, Sh.data(), Sh.size() * sizeof(double));
  if (lam) {
    std::vector<double> l(np);
    gen_eig_device(&budget_, Mh, Sh, np, l.data(), st_);
    std::memcpy(lam, l.data(), np * sizeof(double));
  }
}

}  // namespace sth
