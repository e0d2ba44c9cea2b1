// Dielectric eigensolver: the lowest eigenpairs of chi_bar0 = v^{1/2} chi0 v^{1/2}
// (paper, Section 3: the projective dielectric eigendecomposition, an iterative
// Davidson eigensolver whose products chi0 x are Delta n responses from the
// Sternheimer solves; v the bare Coulomb interaction).
//
// Block Davidson on real grid functions band-limited to the density sphere,
// with the L2 inner product (Omega / N^3) sum_r:
//   * chi_bar0 X: Delta V = v^{1/2} X (full-grid FFT, sqrt(4 pi)/|G|, inverse
//     FFT), Sternheimer solves of every valence band for those Delta V (the
//     solve server of this context), Delta n, then v^{1/2} Delta n;
//   * Rayleigh-Ritz in FP64 on the device (Jacobi eigensolver), Ritz vectors
//     and residuals r_k = chi_bar0 y_k - lambda_k y_k;
//   * the residuals of the unconverged pairs, orthonormalised against the
//     basis (two classical Gram-Schmidt passes), extend it; when the basis
//     would exceed nmax it restarts from the current Ritz vectors.
// Converged when every one of the npdep lowest Ritz pairs has ||r_k|| <= tol.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "engine.hpp"

namespace sth {

namespace {

struct PdepWork {
  long long n3 = 0;
  DevMem V, AV;          // basis and chi_bar0 basis [nmax][n3] real
  DevMem Y, AY, R;       // Ritz vectors, their images, residuals [npdep][n3]
  DevMem DV, DN;         // perturbations / responses of one block [npdep][n3]
  DevMem Z;              // complex FFT scratch [npdep][n3]
  DevMem small, small2;  // [nmax][nmax] doubles
  DevMem hz, evec;       // [nmax][nmax] complex (eigensolver input / vectors)
  DevMem lam;            // [npdep]
};

}  // namespace

void Context::pdep(int id, int npdep, int nmax, double tol, int maxit, double solve_tol,
                   int precision, double* eig_out, double* vec_out, int ptr_kind,
                   hipStream_t user, int* iters, double* max_resid) {
  check_ptr_kind(ptr_kind);
  if (npdep < 1 || nmax < 2 * npdep || nmax > 512 || !(tol > 0.0) || maxit < 1 ||
      !(solve_tol > 0.0) || !eig_out ||
      (precision != STH_FP64 && precision != STH_MIXED && precision != STH_MIXED_BF16)) {
    set_error("pdep: need npdep >= 1, 2 npdep <= nmax <= 512, tol > 0, maxit >= 1, "
              "solve_tol > 0, eig_out, and a valid precision");
    throw Error(STH_E_INVALID);
  }
  // STH_VERBOSE=1: one progress line per iteration on stderr
  const char* ve = std::getenv("STH_VERBOSE");
  const bool verbose = ve && std::atoi(ve) != 0;
  int N = 0, nv = 0, m2d = 0, plan = 0;
  double omega = 0.0, b = 0.0;
  const z64* tw = nullptr;
  PdepWork w;
  {
    std::lock_guard<std::mutex> glk(gpu_mu_);
    STH_HIP_CHECK(hipSetDevice(device_));
    System& s = sys(id);
    if (s.N > kTileMaxN) {
      set_error("pdep: grid %d above %d (full-grid FFT tile does not fit the LDS)", s.N,
                kTileMaxN);
      throw Error(STH_E_INVALID);
    }
    N = s.N;
    nv = s.nv;
    m2d = 4 * s.m2;
    plan = s.g.plan[0];
    tw = s.g.tw64;
    omega = s.omega;
    b = 6.283185307179586477 / s.L;
    prepare_grid_fft(N);
    order_after(user);
    const long long n3 = (long long)N * N * N;
    w.n3 = n3;
    const size_t vb = (size_t)n3 * sizeof(double);
    w.V = DevMem(&budget_, (size_t)nmax * vb);
    w.AV = DevMem(&budget_, (size_t)nmax * vb);
    w.Y = DevMem(&budget_, (size_t)npdep * vb);
    w.AY = DevMem(&budget_, (size_t)npdep * vb);
    w.R = DevMem(&budget_, (size_t)npdep * vb);
    w.DV = DevMem(&budget_, (size_t)npdep * vb);
    w.DN = DevMem(&budget_, (size_t)npdep * vb);
    w.Z = DevMem(&budget_, (size_t)npdep * n3 * sizeof(z64));
    w.small = DevMem(&budget_, (size_t)nmax * nmax * sizeof(double));
    w.small2 = DevMem(&budget_, (size_t)nmax * nmax * sizeof(double));
    w.hz = DevMem(&budget_, (size_t)nmax * nmax * sizeof(z64));
    w.evec = DevMem(&budget_, (size_t)nmax * nmax * sizeof(z64));
    w.lam = DevMem(&budget_, (size_t)npdep * sizeof(double));
  }
  const long long n3 = w.n3;
  const double wt = omega / double(n3);   // L2 weight of a grid point
  double* V = w.V.as<double>();
  double* AV = w.AV.as<double>();
  std::vector<int32_t> bands(nv);
  for (int i = 0; i < nv; ++i) bands[i] = i;

  // out = v^{1/2} in (power 1) or the density-sphere projection of in (power 0)
  auto coulomb = [&](const double* in, int k, double* out, int power) {
    std::lock_guard<std::mutex> glk(gpu_mu_);
    STH_HIP_CHECK(hipSetDevice(device_));
    z64* Z = w.Z.as<z64>();
    launch_real_to_z(in, n3, Z, n3, n3, k, st_);
    launch_grid_fft(N, plan, -1, Z, n3, k, tw, st_);
    launch_coulomb_filter(Z, n3, k, N, m2d, b, power, 1.0 / double(n3), st_);
    launch_grid_fft(N, plan, +1, Z, n3, k, tw, st_);
    launch_z_to_real(Z, n3, out, n3, n3, k, st_);
    STH_HIP_CHECK(hipStreamSynchronize(st_));
  };
  // out = chi_bar0 in for k grid functions (k <= npdep)
  auto apply_chibar = [&](const double* in, int k, double* out) {
    coulomb(in, k, w.DV.as<double>(), 1);
    const sth_solve_opts o{solve_tol, 0, precision, 0};
    const uint64_t t = submit(id, k, w.DV.as<double>(), nv, bands.data(), o, STH_PTR_DEVICE,
                              nullptr);
    if (!wait(t, 1e9)) {
      set_error("pdep: solves did not finish");
      throw Error(STH_E_INTERNAL);
    }
    fetch_drho(t, w.DN.as<double>(), STH_PTR_DEVICE, nullptr);
    release_ticket(t);
    coulomb(w.DN.as<double>(), k, out, 1);
  };
  // orthonormalise vector x against V[0..m) (two classical Gram-Schmidt passes);
  // false if it is numerically in their span
  std::vector<double> hc(nmax);
  auto orth_append = [&](const double* x, int m) -> bool {
    std::lock_guard<std::mutex> glk(gpu_mu_);
    STH_HIP_CHECK(hipSetDevice(device_));
    double* dst = V + (size_t)m * n3;
    STH_HIP_CHECK(hipMemcpyAsync(dst, x, (size_t)n3 * sizeof(double), hipMemcpyDeviceToDevice,
                                 st_));
    double nrm0 = 0.0;
    launch_gram(dst, n3, 1, dst, n3, 1, n3, wt, w.small.as<double>(), st_);
    STH_HIP_CHECK(hipMemcpyAsync(&nrm0, w.small.as<void>(), sizeof(double),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    for (int pass = 0; pass < 2 && m > 0; ++pass) {
      // c_i = <V_i, x>; x -= sum_i c_i V_i
      launch_gram(V, n3, m, dst, n3, 1, n3, wt, w.small.as<double>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(hc.data(), w.small.as<void>(), m * sizeof(double),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      for (int i = 0; i < m; ++i) hc[i] = -hc[i];
      STH_HIP_CHECK(hipMemcpyAsync(w.small2.as<void>(), hc.data(), m * sizeof(double),
                                   hipMemcpyHostToDevice, st_));
      launch_combine(V, n3, m, w.small2.as<double>(), 1, n3, 1.0, dst, n3, st_);
    }
    double nrm = 0.0;
    launch_gram(dst, n3, 1, dst, n3, 1, n3, wt, w.small.as<double>(), st_);
    STH_HIP_CHECK(hipMemcpyAsync(&nrm, w.small.as<void>(), sizeof(double), hipMemcpyDeviceToHost,
                                 st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    if (!(nrm > 1e-16 * nrm0) || !(nrm > 0.0)) return false;   // relative norm below 1e-8
    launch_scale_vec(dst, n3, 1.0 / std::sqrt(nrm), st_);
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    return true;
  };

  // start: seeded white noise projected on the density sphere, orthonormalised
  {
    std::mt19937_64 rng(20220311);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> h((size_t)npdep * n3);
    for (auto& x : h) x = nd(rng);
    {
      std::lock_guard<std::mutex> glk(gpu_mu_);
      STH_HIP_CHECK(hipMemcpyAsync(w.R.as<void>(), h.data(), h.size() * sizeof(double),
                                   hipMemcpyHostToDevice, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
    }
    coulomb(w.R.as<double>(), npdep, w.R.as<double>(), 0);
  }
  int m = 0;
  for (int k = 0; k < npdep; ++k)
    if (orth_append(w.R.as<double>() + (size_t)k * n3, m)) ++m;
  if (m < npdep) {
    set_error("pdep: start block lost rank");
    throw Error(STH_E_INTERNAL);
  }
  apply_chibar(V, m, AV);

  std::vector<double> G((size_t)nmax * nmax), lam, rn(npdep), U((size_t)nmax * npdep);
  std::vector<z64> hz((size_t)nmax * nmax), ev((size_t)nmax * nmax);
  double res = INFINITY;
  int it = 0;
  for (it = 1; it <= maxit; ++it) {
    // Rayleigh-Ritz on span(V[0..m))
    {
      std::lock_guard<std::mutex> glk(gpu_mu_);
      STH_HIP_CHECK(hipSetDevice(device_));
      launch_gram(V, n3, m, AV, n3, m, n3, wt, w.small.as<double>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(G.data(), w.small.as<void>(), (size_t)m * m * sizeof(double),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
          hz[(size_t)i * m + j] = z64{0.5 * (G[(size_t)i * m + j] + G[(size_t)j * m + i]), 0.0};
      STH_HIP_CHECK(hipMemcpyAsync(w.hz.as<void>(), hz.data(), (size_t)m * m * sizeof(z64),
                                   hipMemcpyHostToDevice, st_));
      lam.assign(m, 0.0);
      eig_hermitian_device(&budget_, w.hz.as<z64>(), m, lam.data(), w.evec.as<z64>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(ev.data(), w.evec.as<void>(), (size_t)m * m * sizeof(z64),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      // Ritz coefficients of the npdep lowest pairs (real: the matrix is real symmetric)
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < npdep; ++j) U[(size_t)i * npdep + j] = ev[(size_t)i * m + j].x;
      STH_HIP_CHECK(hipMemcpyAsync(w.small2.as<void>(), U.data(),
                                   (size_t)m * npdep * sizeof(double), hipMemcpyHostToDevice,
                                   st_));
      STH_HIP_CHECK(hipMemcpyAsync(w.lam.as<void>(), lam.data(), npdep * sizeof(double),
                                   hipMemcpyHostToDevice, st_));
      launch_combine(V, n3, m, w.small2.as<double>(), npdep, n3, 0.0, w.Y.as<double>(), n3, st_);
      launch_combine(AV, n3, m, w.small2.as<double>(), npdep, n3, 0.0, w.AY.as<double>(), n3,
                     st_);
      launch_ritz_resid(w.AY.as<double>(), w.Y.as<double>(), n3, w.lam.as<double>(), npdep, n3,
                        w.R.as<double>(), st_);
      launch_gram(w.R.as<double>(), n3, npdep, w.R.as<double>(), n3, npdep, n3, wt,
                  w.small.as<double>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(G.data(), w.small.as<void>(),
                                   (size_t)npdep * npdep * sizeof(double), hipMemcpyDeviceToHost,
                                   st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
    }
    res = 0.0;
    for (int k = 0; k < npdep; ++k) {
      rn[k] = std::sqrt(std::max(G[(size_t)k * npdep + k], 0.0));
      res = std::max(res, rn[k]);
    }
    if (!(res == res)) {
      set_error("pdep: non-finite residual");
      throw Error(STH_E_INTERNAL);
    }
    if (verbose)
      std::fprintf(stderr, "pdep: iteration %d, basis %d, max residual %.3e, lowest %.10f\n", it,
                   m, res, lam[0]);
    if (res <= tol) break;
    if (it == maxit) break;
    // restart from the Ritz vectors when the new directions would not fit
    int nnew = 0;
    for (int k = 0; k < npdep; ++k) nnew += rn[k] > tol;
    if (m + nnew > nmax) {
      std::lock_guard<std::mutex> glk(gpu_mu_);
      STH_HIP_CHECK(hipMemcpyAsync(V, w.Y.as<void>(), (size_t)npdep * n3 * sizeof(double),
                                   hipMemcpyDeviceToDevice, st_));
      STH_HIP_CHECK(hipMemcpyAsync(AV, w.AY.as<void>(), (size_t)npdep * n3 * sizeof(double),
                                   hipMemcpyDeviceToDevice, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      m = npdep;
    }
    const int m0 = m;
    for (int k = 0; k < npdep; ++k)
      if (rn[k] > tol && orth_append(w.R.as<double>() + (size_t)k * n3, m)) ++m;
    if (m == m0) break;   // no new direction: the basis spans the residuals
    apply_chibar(V + (size_t)m0 * n3, m - m0, AV + (size_t)m0 * n3);
  }
  if (iters) *iters = it;
  if (max_resid) *max_resid = res;
  std::memcpy(eig_out, lam.data(), npdep * sizeof(double));
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  if (vec_out)
    copy_out(vec_out, w.Y.as<void>(), (size_t)npdep * n3 * sizeof(double), ptr_kind, st_);
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  order_before(user);
}

}  // namespace sth
