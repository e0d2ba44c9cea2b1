// Batched Lanczos chains of one orbital (paper, Section 3, equation "lanczos"
// and the recurrences before it; the braket of Section 4.3).
//
// For the orbital psi_i of a resident system and nphi real grid functions
// phi_m, chain m starts from u_m = T_S[phi_m psi_i] (the product in real space
// through the plane kernels, as for a right-hand side) and runs, for all chains
// at once as columns,
//   alpha^l = Re <q^l|H q^l>,
//   r = H q^l - alpha^l q^l - beta^l q^{l-1},
//   r -= sum_{k <= l} <q^k|r> q^k        (orthogonalisation against the chain),
//   beta^{l+1} = ||r||,  q^{l+1} = r / beta^{l+1},
// with beta^1 = ||u_m||, q^1 = u_m / beta^1 and H the dual-space operator of the
// solves (FP64).  Then per chain the tridiagonal eigenpairs (d, U; Jacobi on the
// device) and the braket <u_n|q^l_m> for every n, m, l as one matrix product on
// FP64 MFMA (the start vectors against every chain vector).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "engine.hpp"

namespace sth {

void Context::lanczos(int id, int band, int nphi, const double* phi, int ptr_kind, int nsteps,
                      double* alpha, double* beta, double* d, double* U, double* braket,
                      hipStream_t user) {
  check_ptr_kind(ptr_kind);
  if (nphi < 1 || nphi > 256 || nsteps < 1 || nsteps > 200 || !phi || !alpha || !beta) {
    set_error("lanczos: need 1 <= nphi <= 256, 1 <= nsteps <= 200, phi, alpha and beta");
    throw Error(STH_E_INVALID);
  }
  std::lock_guard<std::mutex> glk(gpu_mu_);
  STH_HIP_CHECK(hipSetDevice(device_));
  System& s = sys(id);
  if (band < 0 || band >= s.nv) {
    set_error("lanczos: band %d out of range [0, %d)", band, s.nv);
    throw Error(STH_E_INVALID);
  }
  order_after(user);
  const int n = s.npw, N = s.N, L = nsteps;
  const long long n3 = (long long)N * N * N;
  const size_t vb = (size_t)n * sizeof(z64);
  DevMem dphi(&budget_, (size_t)nphi * n3 * sizeof(double));
  copy_in(dphi.as<void>(), phi, (size_t)nphi * n3 * sizeof(double), ptr_kind, st_);
  std::vector<const double*> pp(nphi);
  for (int m = 0; m < nphi; ++m) pp[m] = dphi.as<const double>() + (size_t)m * n3;
  DevMem potptr = upload(&budget_, pp, st_);
  std::vector<int> src(nphi, band);
  DevMem dsrc = upload(&budget_, src, st_);
  DevMem u0(&budget_, (size_t)nphi * vb), Q(&budget_, (size_t)L * nphi * vb);
  DevMem hq(&budget_, (size_t)nphi * vb), r(&budget_, (size_t)nphi * vb);
  DevMem dots(&budget_, (size_t)nphi * L * sizeof(z64)), adev(&budget_, nphi * sizeof(z64));
  DevMem bdev(&budget_, nphi * sizeof(double));
  HScratch w;
  h_scratch(s, w, nphi);
  const int* ids = w.ids.as<int>();
  z64* U0 = u0.as<z64>();
  z64* QV = Q.as<z64>();
  auto chain = [&](int k) { return QV + (size_t)k * nphi * n; };

  // start vectors u_m = T_S[phi_m psi_band]
  {
    VecSet<z64> sticks{w.sticks.as<z64>(), (long long)N * s.nst};
    launch_copy_vecs({s.W(), (long long)n}, {U0, (long long)n}, dsrc.as<int>(), ids, nphi, n,
                     st_);
    launch_zfft_inv<double, z64>(s.g, {U0, (long long)n}, sticks, ids, nphi, st_);
    launch_plane_local<double>(s.g, sticks, ids, nphi, nullptr,
                               potptr.as<const double* const>(), st_);
    launch_zfft_fwd<double, z64>(s.g, {sticks.base, sticks.stride}, {U0, (long long)n}, ids,
                                 nphi, ZF_PLAIN, {nullptr, 0}, nullptr, st_);
  }
  std::vector<z64> hz(nphi);
  std::vector<double> hb(nphi);
  // norms of the nphi vectors at v -> hb, then bdev
  auto norms = [&](const z64* v) {
    launch_chain_dots(v, 0, n, 1, v, n, nphi, n, dots.as<z64>(), 1, st_);
    STH_HIP_CHECK(hipMemcpyAsync(hz.data(), dots.as<void>(), nphi * sizeof(z64),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    for (int m = 0; m < nphi; ++m) {
      hb[m] = std::sqrt(std::max(hz[m].x, 0.0));
      if (!(hb[m] > 0.0)) {
        set_error("lanczos: chain %d broke down (zero vector)", m);
        throw Error(STH_E_INTERNAL);
      }
    }
    STH_HIP_CHECK(hipMemcpyAsync(bdev.as<void>(), hb.data(), nphi * sizeof(double),
                                 hipMemcpyHostToDevice, st_));
  };
  norms(U0);
  for (int m = 0; m < nphi; ++m) beta[(size_t)m * L] = hb[m];
  launch_chain_div(U0, bdev.as<double>(), nphi, n, chain(0), st_);
  for (int l = 0; l < L; ++l) {
    h_block(s, w, chain(l), hq.as<z64>(), nphi);
    launch_chain_dots(chain(l), 0, n, 1, hq.as<z64>(), n, nphi, n, adev.as<z64>(), 1, st_);
    STH_HIP_CHECK(hipMemcpyAsync(hz.data(), adev.as<void>(), nphi * sizeof(z64),
                                 hipMemcpyDeviceToHost, st_));
    // bdev holds beta^l, the norm that made q^l (unused on the first step)
    launch_lanczos_three_term(hq.as<z64>(), chain(l), l > 0 ? chain(l - 1) : nullptr,
                              adev.as<z64>(), bdev.as<double>(), nphi, n, r.as<z64>(), st_);
    launch_chain_dots(QV, (long long)nphi * n, n, l + 1, r.as<z64>(), n, nphi, n, dots.as<z64>(),
                      L, st_);
    launch_chain_orth(QV, nphi, n, dots.as<z64>(), L, l + 1, r.as<z64>(), st_);
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    for (int m = 0; m < nphi; ++m) alpha[(size_t)m * L + l] = hz[m].x;
    if (l + 1 < L) {
      norms(r.as<z64>());
      for (int m = 0; m < nphi; ++m) beta[(size_t)m * L + l + 1] = hb[m];
      launch_chain_div(r.as<z64>(), bdev.as<double>(), nphi, n, chain(l + 1), st_);
    }
  }
  // tridiagonal eigenpairs per chain (FP64, device Jacobi)
  if (d || U) {
    DevMem T(&budget_, (size_t)L * L * sizeof(z64)), V(&budget_, (size_t)L * L * sizeof(z64));
    std::vector<z64> ht((size_t)L * L), hv((size_t)L * L);
    std::vector<double> ev(L);
    for (int m = 0; m < nphi; ++m) {
      std::fill(ht.begin(), ht.end(), z64{0.0, 0.0});
      for (int l = 0; l < L; ++l) {
        ht[(size_t)l * L + l].x = alpha[(size_t)m * L + l];
        if (l + 1 < L) {
          ht[(size_t)l * L + l + 1].x = beta[(size_t)m * L + l + 1];
          ht[(size_t)(l + 1) * L + l].x = beta[(size_t)m * L + l + 1];
        }
      }
      STH_HIP_CHECK(hipMemcpyAsync(T.as<void>(), ht.data(), ht.size() * sizeof(z64),
                                   hipMemcpyHostToDevice, st_));
      eig_hermitian_device(&budget_, T.as<z64>(), L, ev.data(), V.as<z64>(), st_);
      STH_HIP_CHECK(hipMemcpyAsync(hv.data(), V.as<void>(), hv.size() * sizeof(z64),
                                   hipMemcpyDeviceToHost, st_));
      STH_HIP_CHECK(hipStreamSynchronize(st_));
      if (d) std::memcpy(d + (size_t)m * L, ev.data(), L * sizeof(double));
      if (U)
        for (size_t e = 0; e < hv.size(); ++e) U[(size_t)m * L * L + e] = hv[e].x;
    }
  }
  // braket[n][m][l] = <u_n|q^l_m>: C[c][n] = sum_g conj(u_n[g]) Q_c[g] over the L nphi
  // chain vectors c = l nphi + m (split-K partials, then their fixed-order sum)
  if (braket) {
    const int ncols = L * nphi;
    std::vector<int> cid(ncols);
    std::iota(cid.begin(), cid.end(), 0);
    DevMem dcid = upload(&budget_, cid, st_);
    DevMem part(&budget_, (size_t)s.nsplit * ncols * nphi * sizeof(z64));
    DevMem C(&budget_, (size_t)ncols * nphi * sizeof(z64));
    launch_gemm_ah_b(U0, n, nphi, {QV, (long long)n}, dcid.as<int>(), ncols, n, s.kchunk,
                     part.as<z64>(), st_);
    launch_reduce_parts(part.as<z64>(), s.nsplit, ncols, nphi, nullptr, 1.0, C.as<z64>(), st_);
    std::vector<z64> hc((size_t)ncols * nphi);
    STH_HIP_CHECK(hipMemcpyAsync(hc.data(), C.as<void>(), hc.size() * sizeof(z64),
                                 hipMemcpyDeviceToHost, st_));
    STH_HIP_CHECK(hipStreamSynchronize(st_));
    for (int nn = 0; nn < nphi; ++nn)
      for (int m = 0; m < nphi; ++m)
        for (int l = 0; l < L; ++l) {
          const z64 v = hc[((size_t)l * nphi + m) * nphi + nn];
          const size_t o = (((size_t)nn * nphi + m) * L + l) * 2;
          braket[o] = v.x;
          braket[o + 1] = v.y;
        }
  }
  STH_HIP_CHECK(hipStreamSynchronize(st_));
  order_before(user);
}

}  // namespace sth
