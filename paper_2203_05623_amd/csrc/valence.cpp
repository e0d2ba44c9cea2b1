// Valence eigenpairs of H on the device: block LOBPCG (Knyazev's locally
// optimal block preconditioned conjugate gradient) with FP64 Rayleigh-Ritz.
//
// The paper takes psi_v and eps_v from a ground-state DFT run and uses the
// Davidson method for the dielectric matrix (Section 3); systems given here
// without states get them from this solver.  Per iteration:
//   R = H X - X theta,  W = R / (max(T(G) - theta, 0) + 1),
//   W and the previous update P made orthonormal against [X] and [X, W]
//   (two passes, numerically dependent directions dropped), H W and H P
//   applied explicitly, Rayleigh-Ritz on span[X, W, P], X <- lowest Ritz
//   vectors, P <- their [W, P] component.
// Subspace products are complex GEMMs on the FP64 matrix cores, the small
// eigenproblems run on the device Jacobi solver.  A block of nbands + 8
// vectors is iterated; the lowest nbands must meet the tolerance.
//
// For many bands (3 (nbands + 8) beyond the Jacobi solver's comfortable size)
// the same routine runs Chebyshev-filtered subspace iteration instead (Zhou and
// Saad's filtered Rayleigh-Ritz): Rayleigh-Ritz problems of only nb vectors,
// each iteration a degree-16 filter in the scaled three-term recurrence (15
// block H applications), orthonormalisation, one H application and
// Rayleigh-Ritz.  The filter damps [theta_nb, b] with b an upper bound of the
// spectrum; the block carries 40% guard vectors by default.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "engine.hpp"

namespace sth {

namespace {

constexpr int kLobpcgMaxDim = 2048;   // largest LOBPCG Rayleigh-Ritz problem (3 nb)

// splitmix64 (Steele, Lea and Flood's SplittableRandom finaliser): a counter-based
// generator, so every coefficient of the start block is drawn independently
__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Start block: X[i][k] = (g1 + i g2) / (1 + T_k)^2 with g1, g2 standard normal
// (Box-Muller on two uniform numbers in (0, 1] from the counter i * npw + k)
__global__ void k_random_start(z64* X, int nb, int npw, const double* kin,
                               unsigned long long seed) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nb * npw) return;
  const unsigned long long a = splitmix64(seed ^ (2ull * t)), b = splitmix64(seed ^ (2ull * t + 1));
  const double u1 = ((a >> 11) + 1.0) * 0x1.0p-53, u2 = (b >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double k = kin[t % npw], damp = 1.0 / ((1.0 + k) * (1.0 + k));
  X[t] = z64{r * cos(2.0 * M_PI * u2) * damp, r * sin(2.0 * M_PI * u2) * damp};
}
constexpr int kChebDegree = 16;       // Chebyshev filter degree of the subspace iteration

struct Lobpcg {
  Context& ctx;
  System& s;
  Context::HScratch& hw;
  hipStream_t st;
  int n;            // npw
  int cap;          // max vectors in a block product (3 nb)
  DevMem part, gram, evec, cmat, tmp1, tmp2, scale, norms, ids, theta;
  std::vector<double> hbuf;

  Lobpcg(Context& c, System& sy, Context::HScratch& w, int capv)
      : ctx(c), s(sy), hw(w), st(c.stream()), n(sy.npw), cap(capv) {
    Budget* b = ctx.budget();
    part = DevMem(b, (size_t)s.nsplit * cap * cap * sizeof(z64));
    gram = DevMem(b, (size_t)cap * cap * sizeof(z64));
    evec = DevMem(b, (size_t)cap * cap * sizeof(z64));
    cmat = DevMem(b, (size_t)cap * cap * sizeof(z64));
    tmp1 = DevMem(b, (size_t)cap * n * sizeof(z64));
    tmp2 = DevMem(b, (size_t)cap * n * sizeof(z64));
    scale = DevMem(b, (size_t)cap * sizeof(double));
    norms = DevMem(b, (size_t)cap * sizeof(double));
    theta = DevMem(b, (size_t)cap * sizeof(double));
    ids = DevMem(b, (size_t)cap * sizeof(int));
    std::vector<int> idv(cap);
    std::iota(idv.begin(), idv.end(), 0);
    STH_HIP_CHECK(hipMemcpyAsync(ids.as<void>(), idv.data(), cap * sizeof(int),
                                 hipMemcpyHostToDevice, st));
    STH_HIP_CHECK(hipStreamSynchronize(st));
  }

  const int* id() const { return ids.as<int>(); }

  // G[m][c] = <A_m | B_c>, m < na, c < nb  (row-major na x nb in `gram`)
  void inner(const z64* A, int na, const z64* B, int nbv) {
    launch_gemm_ah_b(A, n, na, {B, (long long)n}, id(), nbv, n, s.kchunk, part.as<z64>(), st);
    launch_reduce_parts(part.as<z64>(), s.nsplit, nbv, na, nullptr, 1.0, gram.as<z64>(), st,
                        true);
  }
  // C[c][m] = -<A_m | B_c>  (layout for combine, with the sign of a projection)
  void inner_neg(const z64* A, int na, const z64* B, int nbv) {
    launch_gemm_ah_b(A, n, na, {B, (long long)n}, id(), nbv, n, s.kchunk, part.as<z64>(), st);
    launch_reduce_parts(part.as<z64>(), s.nsplit, nbv, na, nullptr, -1.0, cmat.as<z64>(), st);
  }
  // out_c = s0 out_c + sum_m A_m C[c][m], c < nc
  void combine(const z64* A, int nm, const z64* C, z64* out, int nc, double s0) {
    launch_gemm_a_c(A, n, nm, C, {out, (long long)n}, id(), nc, n, s0, {nullptr, 0}, nullptr, st);
  }
  void copy(z64* dst, const z64* src, int nv) {
    STH_HIP_CHECK(hipMemcpyAsync(dst, src, (size_t)nv * n * sizeof(z64),
                                 hipMemcpyDeviceToDevice, st));
  }

  // Rows of V (and HV) normalised, made orthogonal to Q (HQ alike), orthonormalised
  // through the eigen-decomposition of their Gram matrix; twice.  Returns the count.
  int orth(z64* V, int nv, z64* HV, const z64* Q, int nq, const z64* HQ) {
    if (nv == 0) return 0;
    std::vector<double> nr(nv), f(nv);
    launch_row_norms(V, nv, n, norms.as<double>(), st);
    STH_HIP_CHECK(hipMemcpyAsync(nr.data(), norms.as<void>(), nv * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
    STH_HIP_CHECK(hipStreamSynchronize(st));
    for (int i = 0; i < nv; ++i) f[i] = nr[i] > 0 ? 1.0 / std::sqrt(nr[i]) : 1.0;
    STH_HIP_CHECK(hipMemcpyAsync(scale.as<void>(), f.data(), nv * sizeof(double),
                                 hipMemcpyHostToDevice, st));
    launch_scale_rows(V, nv, n, scale.as<double>(), st);
    if (HV) launch_scale_rows(HV, nv, n, scale.as<double>(), st);
    for (int pass = 0; pass < 2; ++pass) {
      if (nq > 0) {
        inner_neg(Q, nq, V, nv);                       // C[v][q] = -<q|v>
        combine(Q, nq, cmat.as<z64>(), V, nv, 1.0);   // V -= Q <Q|V>
        if (HV) combine(HQ, nq, cmat.as<z64>(), HV, nv, 1.0);
      }
      inner(V, nv, V, nv);
      std::vector<double> lam(nv);
      eig_hermitian_device(ctx.budget(), gram.as<z64>(), nv, lam.data(), evec.as<z64>(), st);
      const double lmax = std::max(lam[nv - 1], 1e-300);
      int k0 = 0;
      while (k0 < nv && !(lam[k0] > 1e-10 * lmax)) ++k0;
      std::vector<double> is(nv, 0.0);
      for (int k = k0; k < nv; ++k) is[k] = 1.0 / std::sqrt(lam[k]);
      STH_HIP_CHECK(hipMemcpyAsync(scale.as<void>(), is.data(), nv * sizeof(double),
                                   hipMemcpyHostToDevice, st));
      const int nc = nv - k0;
      launch_cols_to_rows(evec.as<z64>(), nv, 0, nv, k0, nc, scale.as<double>(), cmat.as<z64>(),
                          st);
      combine(V, nv, cmat.as<z64>(), tmp1.as<z64>(), nc, 0.0);
      copy(V, tmp1.as<z64>(), nc);
      if (HV) {
        combine(HV, nv, cmat.as<z64>(), tmp1.as<z64>(), nc, 0.0);
        copy(HV, tmp1.as<z64>(), nc);
      }
      nv = nc;
      if (nv == 0) break;
    }
    return nv;
  }

  // Rayleigh-Ritz on the orthonormal rows S[0..m) with HS: Ritz values to th
  // (host, ascending), eigenvectors as columns in `evec`.
  void rr(const z64* S, const z64* HS, int m, std::vector<double>& th) {
    inner(S, m, HS, m);
    th.assign(m, 0.0);
    eig_hermitian_device(ctx.budget(), gram.as<z64>(), m, th.data(), evec.as<z64>(), st);
  }
};

}  // namespace

void Context::valence(const sth_system_desc& d, int nbands, double tol, int maxit,
                      double* eps_out, double* psi_out, int ptr_kind, double* max_resid,
                      int* iters) {
  for (int k : {ptr_kind, d.ptr_kind})
    if (k != STH_PTR_HOST && k != STH_PTR_DEVICE) {
      set_error("ptr_kind must be STH_PTR_HOST (0) or STH_PTR_DEVICE (1), got %d", k);
      throw Error(STH_E_INVALID);
    }
  if (!(d.L > 0) || d.npw <= 0 || !d.miller || !d.vloc_r || d.nproj < 0 ||
      (d.nproj > 0 && (!d.beta || !d.dij))) {
    set_error("valence: invalid system description");
    throw Error(STH_E_INVALID);
  }
  if (d.n != 24 && d.n != 48 && d.n != 72 && d.n != 96 && d.n != 144) {
    set_error("unsupported grid n=%d (supported: 24, 48, 72, 96, 144)", d.n);
    throw Error(STH_E_INVALID);
  }
  // block LOBPCG while its Rayleigh-Ritz problems (3 (nbands + 8)) stay small for
  // the Jacobi eigensolver, Chebyshev-filtered subspace iteration (problems of nb)
  // beyond; STH_VALENCE=lobpcg or chfsi forces one
  const char* va = std::getenv("STH_VALENCE");
  const bool chfsi = va && std::strcmp(va, "chfsi") == 0   ? true
                     : va && std::strcmp(va, "lobpcg") == 0 ? false
                                                            : 3 * (nbands + 8) > kLobpcgMaxDim;
  // guard vectors above the wanted bands: the filter's convergence factor for
  // band nbands is set by the spectral distance to the top of the block
  // (theta_nb, from which the filter damps), so the subspace iteration keeps a
  // fraction STH_CHFSI_GUARD (default 0.4) of extra vectors
  double gfrac = 0.4;
  if (const char* ge = std::getenv("STH_CHFSI_GUARD")) gfrac = std::atof(ge);
  const int guard = chfsi ? std::max(8, int(gfrac * nbands)) : 8;
  const int nb = nbands + guard;
  if (nbands <= 0 || gfrac < 0.0 || (chfsi ? 2 * nb : 3 * nb) > d.npw) {
    set_error("valence: need 0 < 3 (nbands + 8) <= npw (LOBPCG) or 2 (nbands + guard) <= npw "
              "(subspace iteration, guard = max(8, STH_CHFSI_GUARD x nbands))");
    throw Error(STH_E_INVALID);
  }
  if (maxit <= 0) maxit = 500;
  // STH_VERBOSE=1: one progress line per iteration on stderr (long eigensolves)
  const char* ve = std::getenv("STH_VERBOSE");
  const bool verbose = ve && std::atoi(ve) != 0;
  const auto t_start = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System s;
  StickBuild sb = setup_geometry(s, d, 0);
  if (verbose)
    std::fprintf(stderr, "valence: %d vectors (%d bands + %d guard), set-up %.1f s\n", nb, nbands,
                 guard,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
  const int n = s.npw;
  HScratch hw;
  h_scratch(s, hw, std::min(nb, 256));
  Lobpcg L(*this, s, hw, chfsi ? nb : 3 * nb);
  const size_t vb = (size_t)n * sizeof(z64);
  const int nblock = chfsi ? 1 : 3;   // blocks of nb vectors in S and HS
  DevMem S(&budget_, nblock * (size_t)nb * vb), HS(&budget_, nblock * (size_t)nb * vb);
  DevMem P, HP;
  if (!chfsi) {
    P = DevMem(&budget_, (size_t)nb * vb);
    HP = DevMem(&budget_, (size_t)nb * vb);
  }
  z64* X = S.as<z64>();
  z64* HX = HS.as<z64>();

  // start: seeded random vectors damped at high kinetic energy, drawn on the device
  hipLaunchKernelGGL(k_random_start, dim3(unsigned(((long long)nb * n + 255) / 256)), dim3(256),
                     0, st_, X, nb, n, s.d_kin.as<double>(), 7ull);
  STH_HIP_CHECK(hipGetLastError());
  if (L.orth(X, nb, nullptr, nullptr, 0, nullptr) != nb) {
    set_error("valence: degenerate start block");
    throw Error(STH_E_INTERNAL);
  }
  h_block(s, hw, X, HX, nb);
  int np = 0;
  std::vector<double> th, rn(nb);
  double res = INFINITY;
  int it = 0;
  auto progress = [&]() {
    if (verbose)
      std::fprintf(stderr, "valence: iteration %d, max residual %.3e, %.1f s\n", it, res,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start)
                       .count());
    if (!(res == res)) {
      set_error("valence: non-finite residual");
      throw Error(STH_E_INTERNAL);
    }
  };
  DevMem Yb, Zb, HY;   // Chebyshev filter blocks (ChFSI only)
  if (chfsi) {
    // Chebyshev-filtered subspace iteration (Zhou & Saad): each iteration applies
    // the degree-kChebDegree Chebyshev polynomial of H that is small on
    // [theta_nb, upper bound of the spectrum] and large below it, in its scaled
    // three-term form, then orthonormalises and does Rayleigh-Ritz on the nb
    // filtered vectors.
    Yb = DevMem(&budget_, (size_t)nb * vb);
    Zb = DevMem(&budget_, (size_t)nb * vb);
    HY = DevMem(&budget_, (size_t)nb * vb);
    const long long nel = (long long)nb * n;
    // upper bound of the spectrum: a few Lanczos steps on one vector; Gershgorin
    // of their tridiagonal matrix plus the last residual norm
    double bup = 0.0;
    {
      constexpr int K = 12;
      std::mt19937_64 rng(11);
      std::normal_distribution<double> nd(0.0, 1.0);
      std::vector<z64> v(n), w(n), vp(n, z64{0.0, 0.0});
      double nrm = 0.0;
      for (auto& x : v) {
        x = z64{nd(rng), nd(rng)};
        nrm += x.x * x.x + x.y * x.y;
      }
      for (auto& x : v) x = z64{x.x / std::sqrt(nrm), x.y / std::sqrt(nrm)};
      std::vector<double> al(K), be(K + 1, 0.0);
      int kk = K;
      z64* dv = Yb.as<z64>();
      z64* dw = Zb.as<z64>();
      for (int k = 0; k < K; ++k) {
        STH_HIP_CHECK(hipMemcpyAsync(dv, v.data(), vb, hipMemcpyHostToDevice, st_));
        h_block(s, hw, dv, dw, 1);
        STH_HIP_CHECK(hipMemcpyAsync(w.data(), dw, vb, hipMemcpyDeviceToHost, st_));
        STH_HIP_CHECK(hipStreamSynchronize(st_));
        double a = 0.0;
        for (int g = 0; g < n; ++g) a += v[g].x * w[g].x + v[g].y * w[g].y;
        double b2 = 0.0;
        for (int g = 0; g < n; ++g) {
          w[g].x -= a * v[g].x + be[k] * vp[g].x;
          w[g].y -= a * v[g].y + be[k] * vp[g].y;
          b2 += w[g].x * w[g].x + w[g].y * w[g].y;
        }
        al[k] = a;
        be[k + 1] = std::sqrt(b2);
        if (!(be[k + 1] > 1e-12 * std::fabs(a))) {   // invariant subspace: T is exact
          kk = k + 1;
          break;
        }
        vp = v;
        for (int g = 0; g < n; ++g) v[g] = z64{w[g].x / be[k + 1], w[g].y / be[k + 1]};
      }
      // Gershgorin bound of the kk x kk tridiagonal matrix, plus the norm of the
      // last residual
      double gersh = -INFINITY;
      for (int k = 0; k < kk; ++k)
        gersh = std::max(gersh, al[k] + be[k] + (k + 1 < kk ? be[k + 1] : 0.0));
      bup = gersh + be[kk];
    }
    z64* bufs[3] = {S.as<z64>(), Yb.as<z64>(), Zb.as<z64>()};
    auto rr_rotate = [&]() {
      L.rr(X, HX, nb, th);
      launch_cols_to_rows(L.evec.as<z64>(), nb, 0, nb, 0, nb, nullptr, L.cmat.as<z64>(), st_);
      L.combine(X, nb, L.cmat.as<z64>(), L.tmp1.as<z64>(), nb, 0.0);
      L.combine(HX, nb, L.cmat.as<z64>(), L.tmp2.as<z64>(), nb, 0.0);
      L.copy(X, L.tmp1.as<z64>(), nb);
      L.copy(HX, L.tmp2.as<z64>(), nb);
    };
    // per-phase wall time of an iteration (progress lines only: the stream is
    // drained before each reading)
    auto t_lap = std::chrono::steady_clock::now();
    auto lap = [&]() {
      if (!verbose) return 0.0;
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      const auto t = std::chrono::steady_clock::now();
      const double d = std::chrono::duration<double>(t - t_lap).count();
      t_lap = t;
      return d;
    };
    rr_rotate();
    double a0 = th[0];
    for (; it < maxit; ++it) {
      STH_HIP_CHECK(hipMemcpyAsync(L.theta.as<void>(), th.data(), nb * sizeof(double),
                                   hipMemcpyHostToDevice, st_));
      z64* spare[2];
      for (int b = 0, k = 0; b < 3; ++b)
        if (bufs[b] != X) spare[k++] = bufs[b];
      launch_resid_precond(s.g, X, HX, L.theta.as<double>(), nb, spare[0],
                           L.norms.as<double>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(rn.data(), L.norms.as<void>(), nb * sizeof(double),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      res = 0.0;
      for (int i = 0; i < nbands; ++i) res = std::max(res, std::sqrt(rn[i]));
      progress();
      if (res <= tol) break;
      const double a = th[nb - 1];
      const double e = 0.5 * (bup - a), c = 0.5 * (bup + a);
      if (!(e > 0.0)) {
        set_error("valence: empty filter interval (upper bound %.6f, theta_nb %.6f)", bup, a);
        throw Error(STH_E_INTERNAL);
      }
      lap();
      double sigma = e / (a0 - c);
      const double tau = 2.0 / sigma;
      z64* xp = X;          // previous filtered block
      z64* yc = spare[0];   // current
      z64* yn = spare[1];   // next
      launch_block_axpbypcz(nel, sigma / e, HX, -c * sigma / e, X, 0.0, nullptr, yc, st_);
      for (int k = 2; k <= kChebDegree; ++k) {
        h_block(s, hw, yc, HY.as<z64>(), nb);
        const double sn = 1.0 / (tau - sigma);
        launch_block_axpbypcz(nel, 2.0 * sn / e, HY.as<z64>(), -2.0 * c * sn / e, yc,
                              -sigma * sn, xp, yn, st_);
        z64* t = xp;
        xp = yc;
        yc = yn;
        yn = t;
        sigma = sn;
      }
      const double t_f = lap();
      if (L.orth(yc, nb, nullptr, nullptr, 0, nullptr) != nb) {
        set_error("valence: filtered block lost rank");
        throw Error(STH_E_INTERNAL);
      }
      const double t_o = lap();
      X = yc;
      h_block(s, hw, X, HX, nb);
      const double t_h = lap();
      rr_rotate();
      const double t_r = lap();
      if (verbose)
        std::fprintf(stderr, "valence: filter %.2f s, orthonormalisation %.2f s, H %.2f s, "
                             "Rayleigh-Ritz %.2f s\n", t_f, t_o, t_h, t_r);
      a0 = std::min(a0, th[0]);
    }
  }
  for (; !chfsi && it < maxit; ++it) {
    if (it > 0 && it % 8 == 0) h_block(s, hw, X, HX, nb);   // refresh the carried products
    if (L.orth(X, nb, HX, nullptr, 0, nullptr) != nb) {
      set_error("valence: block lost rank");
      throw Error(STH_E_INTERNAL);
    }
    // Rayleigh-Ritz on X
    L.rr(X, HX, nb, th);
    launch_cols_to_rows(L.evec.as<z64>(), nb, 0, nb, 0, nb, nullptr, L.cmat.as<z64>(), st_);
    L.combine(X, nb, L.cmat.as<z64>(), L.tmp1.as<z64>(), nb, 0.0);
    L.combine(HX, nb, L.cmat.as<z64>(), L.tmp2.as<z64>(), nb, 0.0);
    L.copy(X, L.tmp1.as<z64>(), nb);
    L.copy(HX, L.tmp2.as<z64>(), nb);
    STH_HIP_CHECK(hipMemcpyAsync(L.theta.as<void>(), th.data(), nb * sizeof(double),
                                 hipMemcpyHostToDevice, st_));
    // residuals and preconditioned directions W (rows nb..2nb of S)
    z64* Wd = X + (size_t)nb * n;
    launch_resid_precond(s.g, X, HX, L.theta.as<double>(), nb, Wd, L.norms.as<double>(), st_);
    STH_HIP_CHECK(hipMemcpyAsync(rn.data(), L.norms.as<void>(), nb * sizeof(double),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    res = 0.0;
    for (int i = 0; i < nbands; ++i) res = std::max(res, std::sqrt(rn[i]));
    progress();
    if (res <= tol) break;
    const int nw = L.orth(Wd, nb, nullptr, X, nb, nullptr);
    h_block(s, hw, Wd, HX + (size_t)nb * n, nw);
    int m = nb + nw;
    if (np > 0) {
      z64* Pd = X + (size_t)m * n;
      L.copy(Pd, P.as<z64>(), np);
      const int np2 = L.orth(Pd, np, nullptr, X, m, nullptr);
      h_block(s, hw, Pd, HX + (size_t)m * n, np2);
      m += np2;
    }
    // Rayleigh-Ritz on [X, W, P]
    L.rr(X, HX, m, th);
    launch_cols_to_rows(L.evec.as<z64>(), m, 0, m, 0, nb, nullptr, L.cmat.as<z64>(), st_);
    L.combine(X, m, L.cmat.as<z64>(), L.tmp1.as<z64>(), nb, 0.0);
    L.combine(HX, m, L.cmat.as<z64>(), L.tmp2.as<z64>(), nb, 0.0);
    // P <- [W, P] part of the new X
    launch_cols_to_rows(L.evec.as<z64>(), m, nb, m - nb, 0, nb, nullptr, L.cmat.as<z64>(), st_);
    L.combine(X + (size_t)nb * n, m - nb, L.cmat.as<z64>(), P.as<z64>(), nb, 0.0);
    L.combine(HX + (size_t)nb * n, m - nb, L.cmat.as<z64>(), HP.as<z64>(), nb, 0.0);
    np = nb;
    L.copy(X, L.tmp1.as<z64>(), nb);
    L.copy(HX, L.tmp2.as<z64>(), nb);
  }
  if (max_resid) *max_resid = res;
  if (iters) *iters = it;
  if (!(res <= tol)) {
    set_error("valence: not converged after %d iterations (max residual %.3e)", it, res);
    throw Error(STH_E_INTERNAL);
  }
  // outputs: eigenvalues and vectors in caller order
  DevMem out(&budget_, (size_t)nbands * vb);
  launch_permute_out(X, n, out.as<z64>(), n, s.d_perm.as<int>(), n, nbands, st_);
  if (ptr_kind == STH_PTR_DEVICE) {
    STH_HIP_CHECK(hipMemcpyAsync(eps_out, th.data(), nbands * sizeof(double),
                                 hipMemcpyHostToDevice, st_));
    STH_HIP_CHECK(hipMemcpyAsync(psi_out, out.as<void>(), (size_t)nbands * vb,
                                 hipMemcpyDeviceToDevice, st_));
  } else {
    std::memcpy(eps_out, th.data(), nbands * sizeof(double));
    STH_HIP_CHECK(hipMemcpyAsync(psi_out, out.as<void>(), (size_t)nbands * vb,
                                 hipMemcpyDeviceToHost, st_));
  }
  STH_HIP_CHECK(hipStreamSynchronize(st_));
}

}  // namespace sth
