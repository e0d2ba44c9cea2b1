// Vector kernels of the batched preconditioned conjugate gradient (paper,
// Section 3: each Sternheimer equation is solved by a preconditioned CG,
// independently per perturbation and orbital).  FP64 state and reductions.
//
// Reductions are deterministic: every workgroup writes one partial per chunk
// of 1024 coefficients (wavefront shuffles, then LDS across the 4 waves in a
// fixed order) and a per-slot scalar kernel sums the partials in order.
//
// Preconditioner (the paper only says "preconditioned"): the Teter-Payne-Allan
// diagonal K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4),
// x = T(G) / max(E_kin(v), 0.1 Ha), with E_kin(v) = <psi_v|T|psi_v>.
#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

constexpr int CTHR = 256;
constexpr int CHUNK = 1024;

__device__ inline double tpa(double kin, double ekin) {
  const double x = kin / fmax(ekin, 0.1);
  const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
  return num / (num + 16.0 * x * x * x * x);
}

// ||r||^2 at which a run of the recurrence stops and the true residual is taken:
// the final target for FP64 solves; for the FP32 inner runs of a mixed solve a
// fixed reduction of the residual the run started from (defect correction).
__device__ inline double inner_target2(double final2, double start2, int prec) {
  if (!prec) return final2;
  return fmax(final2, MIXED_INNER_REDUCTION * MIXED_INNER_REDUCTION * start2);
}

// block-wide sum of two values, result valid in thread 0; fixed order
__device__ inline void block_sum2(double& a, double& b) {
  __shared__ double sa[CTHR / 64], sb[CTHR / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sa[0];
    b = sb[0];
    for (int i = 1; i < CTHR / 64; ++i) {
      a += sa[i];
      b += sb[i];
    }
  }
}

__global__ __launch_bounds__(CTHR) void k_cg_init(GridDev g, VecSet<const z64> b, VecSet<z64> x,
                                                  VecSet<z64> r, VecSet<z64> p,
                                                  const int* slots, const double* ekin_slot,
                                                  double* part2) {
  const int c = blockIdx.y, slot = slots[c];
  const double ek = ekin_slot[slot];
  const z64* bb = b.base + slot * b.stride;
  z64* xx = x.base + slot * x.stride;
  z64* rr = r.base + slot * r.stride;
  z64* pp = p.base + slot * p.stride;
  double s1 = 0.0, s2 = 0.0;
  const int e0 = blockIdx.x * CHUNK;
  for (int e = e0 + threadIdx.x; e < min(e0 + CHUNK, g.npw); e += CTHR) {
    const z64 v = bb[e];
    const double k = tpa(g.kin[e], ek);
    xx[e] = z64{0.0, 0.0};
    rr[e] = v;
    pp[e] = z64{k * v.x, k * v.y};
    s1 += k * (v.x * v.x + v.y * v.y);
    s2 += v.x * v.x + v.y * v.y;
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 0] = s1;
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

__global__ void k_cg_init_scalars(const double* part2, int nchunk, const int* slots, int ncols,
                                  SlotState s) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int slot = slots[c];
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nchunk; ++i) {
    a += part2[((long long)c * nchunk + i) * 2 + 0];
    b += part2[((long long)c * nchunk + i) * 2 + 1];
  }
  s.rho[slot] = a;
  s.bnorm2[slot] = b;
  s.rnorm2[slot] = b;
  s.alpha[slot] = 0.0;
  s.beta[slot] = 0.0;
  s.iters[slot] = 0;
  s.tgt2[slot] = inner_target2(s.tol[slot] * s.tol[slot] * b, b, s.prec[slot]);
  s.status[slot] = (b > 0.0) ? SLOT_ACTIVE : (b == 0.0 ? SLOT_DONE : SLOT_NAN);
}

// alpha = rho / <p, A p> per column: one wavefront per column sums the per-tile
// partials (lane l takes tiles l, l + 64, ...; then a fixed butterfly order).
__global__ __launch_bounds__(64) void k_cg_alpha(const double* dots, int ntile,
                                                 const int* slots, int ncols, SlotState s) {
  const int c = blockIdx.x;
  if (c >= ncols) return;
  const int slot = slots[c];
  const int l = threadIdx.x;
  double pq = 0.0;
  for (int t = l; t < ntile; t += 64) pq += dots[(long long)c * ntile + t];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pq += __shfl_xor(pq, o);
  if (l != 0) return;
  if (s.status[slot] != SLOT_ACTIVE) {
    s.alpha[slot] = 0.0;
    return;
  }
  if (pq > 0.0) {
    s.alpha[slot] = s.rho[slot] / pq;
  } else {
    s.alpha[slot] = 0.0;
    s.status[slot] = (pq != pq) ? SLOT_NAN : SLOT_BREAKDOWN;
  }
}

__global__ __launch_bounds__(CTHR) void k_cg_update_xr(GridDev g, VecSet<z64> x, VecSet<z64> r,
                                                       VecSet<const z64> p, VecSet<const z64> q,
                                                       const int* slots, SlotState s,
                                                       double* part2) {
  const int c = blockIdx.y, slot = slots[c];
  const bool active = s.status[slot] == SLOT_ACTIVE;
  const double al = s.alpha[slot], ek = s.ekin[slot];
  z64* xx = x.base + slot * x.stride;
  z64* rr = r.base + slot * r.stride;
  const z64* pp = p.base + slot * p.stride;
  const z64* qq = q.base + slot * q.stride;
  double s1 = 0.0, s2 = 0.0;
  const int e0 = blockIdx.x * CHUNK;
  if (active) {
    for (int e = e0 + threadIdx.x; e < min(e0 + CHUNK, g.npw); e += CTHR) {
      const z64 pv = pp[e], qv = qq[e];
      z64 xv = xx[e], rv = rr[e];
      xv.x += al * pv.x;
      xv.y += al * pv.y;
      rv.x -= al * qv.x;
      rv.y -= al * qv.y;
      xx[e] = xv;
      rr[e] = rv;
      const double k = tpa(g.kin[e], ek);
      const double n2 = rv.x * rv.x + rv.y * rv.y;
      s1 += k * n2;
      s2 += n2;
    }
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 0] = s1;
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

__global__ void k_cg_beta(const double* part2, int nchunk, const int* slots, int ncols,
                          SlotState s) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int slot = slots[c];
  if (s.status[slot] != SLOT_ACTIVE) {
    s.beta[slot] = 0.0;
    return;
  }
  double rz = 0.0, rr = 0.0;
  for (int i = 0; i < nchunk; ++i) {
    rz += part2[((long long)c * nchunk + i) * 2 + 0];
    rr += part2[((long long)c * nchunk + i) * 2 + 1];
  }
  const int it = s.iters[slot] + 1;
  s.iters[slot] = it;
  s.rnorm2[slot] = rr;
  if (rr != rr) {
    s.status[slot] = SLOT_NAN;
    s.beta[slot] = 0.0;
  } else if (rr <= s.tgt2[slot]) {
    s.status[slot] = SLOT_CHECK;
    s.beta[slot] = 0.0;
  } else if (it >= s.maxit[slot]) {
    s.status[slot] = SLOT_MAXIT;
    s.beta[slot] = 0.0;
  } else {
    s.beta[slot] = rz / s.rho[slot];
    s.rho[slot] = rz;
  }
}

__global__ __launch_bounds__(CTHR) void k_cg_update_p(GridDev g, VecSet<const z64> r,
                                                      VecSet<z64> p, const int* slots,
                                                      SlotState s) {
  const int c = blockIdx.y, slot = slots[c];
  if (s.status[slot] != SLOT_ACTIVE) return;
  const double be = s.beta[slot], ek = s.ekin[slot];
  const z64* rr = r.base + slot * r.stride;
  z64* pp = p.base + slot * p.stride;
  const int e0 = blockIdx.x * CHUNK;
  for (int e = e0 + threadIdx.x; e < min(e0 + CHUNK, g.npw); e += CTHR) {
    const double k = tpa(g.kin[e], ek);
    const z64 rv = rr[e];
    z64 pv = pp[e];
    pv.x = k * rv.x + be * pv.x;
    pv.y = k * rv.y + be * pv.y;
    pp[e] = pv;
  }
}

__global__ __launch_bounds__(CTHR) void k_cg_true_resid(GridDev g, VecSet<const z64> b,
                                                        VecSet<const z64> q, VecSet<z64> r,
                                                        const int* slots,
                                                        const double* ekin_slot,
                                                        double* part2) {
  const int c = blockIdx.y, slot = slots[c];
  const double ek = ekin_slot[slot];
  const z64* bb = b.base + slot * b.stride;
  const z64* qq = q.base + slot * q.stride;
  z64* rr = r.base + slot * r.stride;
  double s1 = 0.0, s2 = 0.0;
  const int e0 = blockIdx.x * CHUNK;
  for (int e = e0 + threadIdx.x; e < min(e0 + CHUNK, g.npw); e += CTHR) {
    const z64 bv = bb[e], qv = qq[e];
    const z64 rv = {bv.x - qv.x, bv.y - qv.y};
    rr[e] = rv;
    const double n2 = rv.x * rv.x + rv.y * rv.y;
    s1 += tpa(g.kin[e], ek) * n2;
    s2 += n2;
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) {
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 0] = s1;
    part2[((long long)c * gridDim.x + blockIdx.x) * 2 + 1] = s2;
  }
}

// After a true residual: DONE if it meets tol, else restart the recurrence on it
// (rho = <r, K r>, beta = 0, so the next p-update sets p = K r).  With
// final_only the slot has already stopped (MAXIT or BREAKDOWN): only its
// residual norm is replaced by the true one.
__global__ void k_cg_check_true(const double* part2, int nchunk, const int* slots, int ncols,
                                SlotState s, int final_only) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int slot = slots[c];
  double rz = 0.0, rr = 0.0;
  for (int i = 0; i < nchunk; ++i) {
    rz += part2[((long long)c * nchunk + i) * 2 + 0];
    rr += part2[((long long)c * nchunk + i) * 2 + 1];
  }
  s.rnorm2[slot] = rr;
  s.beta[slot] = 0.0;
  if (final_only) {
    if (rr != rr) s.status[slot] = SLOT_NAN;
    return;
  }
  if (rr != rr) {
    s.status[slot] = SLOT_NAN;
  } else if (rr <= s.tol[slot] * s.tol[slot] * s.bnorm2[slot]) {
    s.status[slot] = SLOT_DONE;
  } else if (s.iters[slot] >= s.maxit[slot]) {
    s.status[slot] = SLOT_MAXIT;
  } else {
    s.status[slot] = SLOT_ACTIVE;
    s.rho[slot] = rz;
    s.tgt2[slot] = inner_target2(s.tol[slot] * s.tol[slot] * s.bnorm2[slot], rr, s.prec[slot]);
  }
}

__global__ void k_copy_vecs(VecSet<const z64> src, VecSet<z64> dst, const int* ss,
                            const int* sd, int n) {
  const int c = blockIdx.y;
  const z64* a = src.base + (ss ? ss[c] : c) * src.stride;
  z64* b = dst.base + (sd ? sd[c] : c) * dst.stride;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    b[e] = a[e];
}

__global__ void k_scale_vecs(VecSet<z64> v, const int* slots, int n, double s) {
  z64* a = v.base + (slots ? slots[blockIdx.y] : blockIdx.y) * v.stride;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    a[e].x *= s;
    a[e].y *= s;
  }
}

// dst[c][perm[e]] = src[c][e]   (perm maps caller order -> internal order)
__global__ void k_permute_in(const z64* src, long long ss, z64* dst, long long ds, const int* perm,
                             int n) {
  const int c = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    dst[c * ds + perm[e]] = src[c * ss + e];
}

// dst[c][e] = src[c][perm[e]]
__global__ void k_permute_out(const z64* src, long long ss, z64* dst, long long ds,
                              const int* perm, int n) {
  const int c = blockIdx.y;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
    dst[c * ds + e] = src[c * ss + perm[e]];
}

__global__ void k_z64_to_z32(const z64* s, z32* d, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    d[i] = z32{float(s[i].x), float(s[i].y)};
}

__global__ void k_to_f32(const double* s, float* d, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    d[i] = float(s[i]);
}

__global__ __launch_bounds__(CTHR) void k_row_norms(const z64* v, int n, double* out) {
  const z64* a = v + (long long)blockIdx.x * n;
  double s1 = 0.0, s2 = 0.0;
  for (int e = threadIdx.x; e < n; e += CTHR) s1 += a[e].x * a[e].x + a[e].y * a[e].y;
  block_sum2(s1, s2);
  if (threadIdx.x == 0) out[blockIdx.x] = s1;
}

__global__ void k_scale_rows(z64* v, int n, const double* f) {
  z64* a = v + (long long)blockIdx.y * n;
  const double s = f[blockIdx.y];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    a[e].x *= s;
    a[e].y *= s;
  }
}

__global__ __launch_bounds__(CTHR) void k_resid_precond(GridDev g, const z64* X, const z64* HX,
                                                        const double* theta, z64* W,
                                                        double* out) {
  const int i = blockIdx.x;
  const long long o = (long long)i * g.npw;
  const double th = theta[i];
  double s1 = 0.0, s2 = 0.0;
  for (int e = threadIdx.x; e < g.npw; e += CTHR) {
    const z64 x = X[o + e], h = HX[o + e];
    const z64 r = {h.x - th * x.x, h.y - th * x.y};
    const double d = 1.0 / (fmax(g.kin[e] - th, 0.0) + 1.0);
    W[o + e] = z64{r.x * d, r.y * d};
    s1 += r.x * r.x + r.y * r.y;
  }
  block_sum2(s1, s2);
  if (threadIdx.x == 0) out[i] = s1;
}

__global__ void k_cols_to_rows(const z64* U, int ldu, int m0, int nm, int col0, int nc,
                               const double* scale, z64* C) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nc * nm) return;
  const int c = int(t / nm), m = int(t % nm);
  const double f = scale ? scale[col0 + c] : 1.0;
  const z64 u = U[(long long)(m0 + m) * ldu + col0 + c];
  C[t] = z64{u.x * f, u.y * f};
}

inline dim3 vec_grid(int npw, int ncols) { return dim3(cg_chunks(npw), ncols); }
inline dim3 scalar_grid(int ncols) { return dim3((ncols + 127) / 128); }

}  // namespace

void launch_cg_init(const GridDev& g, VecSet<const z64> b, VecSet<z64> x, VecSet<z64> r,
                    VecSet<z64> p, const int* slots, int ncols, const double* ekin,
                    double* part2, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_init, vec_grid(g.npw, ncols), dim3(CTHR), 0, st, g, b, x, r, p, slots,
                     ekin, part2);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_init_scalars(const double* part2, int nchunk, const int* slots, int ncols,
                            SlotState s, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_init_scalars, scalar_grid(ncols), dim3(128), 0, st, part2, nchunk,
                     slots, ncols, s);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_alpha(const double* dots, int ntile, const int* slots, int ncols, SlotState s,
                     hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_alpha, dim3(ncols), dim3(64), 0, st, dots, ntile, slots, ncols, s);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_update_xr(const GridDev& g, VecSet<z64> x, VecSet<z64> r, VecSet<const z64> p,
                         VecSet<const z64> q, const int* slots, int ncols, SlotState s,
                         double* part2, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_update_xr, vec_grid(g.npw, ncols), dim3(CTHR), 0, st, g, x, r, p, q,
                     slots, s, part2);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_beta(const double* part2, int nchunk, const int* slots, int ncols, SlotState s,
                    hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_beta, scalar_grid(ncols), dim3(128), 0, st, part2, nchunk, slots,
                     ncols, s);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_update_p(const GridDev& g, VecSet<const z64> r, VecSet<z64> p, const int* slots,
                        int ncols, SlotState s, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_update_p, vec_grid(g.npw, ncols), dim3(CTHR), 0, st, g, r, p, slots,
                     s);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_true_resid(const GridDev& g, VecSet<const z64> b, VecSet<const z64> q,
                          VecSet<z64> r, const int* slots, int ncols, const double* ekin_slot,
                          double* part2, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_true_resid, vec_grid(g.npw, ncols), dim3(CTHR), 0, st, g, b, q, r,
                     slots, ekin_slot, part2);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cg_check_true(const double* part2, int nchunk, const int* slots, int ncols,
                          SlotState s, hipStream_t st, bool final_only) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_cg_check_true, scalar_grid(ncols), dim3(128), 0, st, part2, nchunk, slots,
                     ncols, s, int(final_only));
  STH_HIP_CHECK(hipGetLastError());
}

void launch_copy_vecs(VecSet<const z64> src, VecSet<z64> dst, const int* slots_src,
                      const int* slots_dst, int ncols, int n, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_copy_vecs, dim3((n + 1023) / 1024, ncols), dim3(256), 0, st, src, dst,
                     slots_src, slots_dst, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_scale_vecs(VecSet<z64> v, const int* slots, int ncols, int n, double s,
                       hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_scale_vecs, dim3((n + 1023) / 1024, ncols), dim3(256), 0, st, v, slots, n,
                     s);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_permute_in(const z64* src, long long sstride, z64* dst, long long dstride,
                       const int* perm, int n, int ncols, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_permute_in, dim3((n + 1023) / 1024, ncols), dim3(256), 0, st, src,
                     sstride, dst, dstride, perm, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_permute_out(const z64* src, long long sstride, z64* dst, long long dstride,
                        const int* perm, int n, int ncols, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  hipLaunchKernelGGL(k_permute_out, dim3((n + 1023) / 1024, ncols), dim3(256), 0, st, src,
                     sstride, dst, dstride, perm, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_row_norms(const z64* v, int nvec, int n, double* out, hipStream_t st) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_row_norms, dim3(nvec), dim3(CTHR), 0, st, v, n, out);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_scale_rows(z64* v, int nvec, int n, const double* f, hipStream_t st) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_scale_rows, dim3((n + 1023) / 1024, nvec), dim3(256), 0, st, v, n, f);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_resid_precond(const GridDev& g, const z64* X, const z64* HX, const double* theta,
                          int nvec, z64* W, double* out, hipStream_t st) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_resid_precond, dim3(nvec), dim3(CTHR), 0, st, g, X, HX, theta, W, out);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_cols_to_rows(const z64* U, int ldu, int m0, int nm, int col0, int nc,
                         const double* scale, z64* C, hipStream_t st) {
  const long long n = (long long)nc * nm;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cols_to_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, U, ldu,
                     m0, nm, col0, nc, scale, C);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_z64_to_z32(const z64* src, z32* dst, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_z64_to_z32, dim3(1024), dim3(256), 0, st, src, dst, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_to_f32(const double* src, float* dst, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, st, src, dst, n);
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
