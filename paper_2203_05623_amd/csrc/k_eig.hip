// Dense Hermitian eigensolver for the small Rayleigh-Ritz problems of the path
// (valence LOBPCG subspace, chi0 block), FP64 on the device.
//
// Cyclic two-sided Jacobi with a round-robin (tournament) ordering: every
// round rotates n/2 disjoint index pairs at once, so a round is two fully
// parallel kernels (columns, then rows).  For a pair (p, q) with
// A_pq = |b| e^{i phi}, the unitary U = diag(1, e^{-i phi}) R, R the real
// Jacobi rotation of [[A_pp, |b|], [|b|, A_qq]] (Golub & Van Loan, symmetric
// Schur decomposition), zeroes A_pq in U^H A U.  Eigenvectors accumulate in
// V <- V U.  Matrices are row-major n x n complex (z64).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "engine.hpp"

namespace sth {

namespace {

struct Rot {
  double c, s, cph, sph;   // U = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
};

__global__ void k_jac_params(const z64* A, int n, const int2* pairs, int np, Rot* rot) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const int p = pairs[k].x, q = pairs[k].y;
  Rot r{1.0, 0.0, 1.0, 0.0};
  if (p < n && q < n) {
    const z64 b = A[(long long)p * n + q];
    const double ab = hypot(b.x, b.y);
    const double a = A[(long long)p * n + p].x, d = A[(long long)q * n + q].x;
    if (ab > 1e-300 && ab > 1e-18 * (fabs(a) + fabs(d))) {
      const double tau = (d - a) / (2.0 * ab);
      const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      r.c = 1.0 / sqrt(1.0 + t * t);
      r.s = t * r.c;
      r.cph = b.x / ab;
      r.sph = b.y / ab;
    }
  }
  rot[k] = r;
}

// X <- X U on columns (p, q) for every row; applied to A and V
__global__ void k_jac_cols(z64* A, z64* V, int n, const int2* pairs, int np, const Rot* rot) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = int(t / n), i = int(t % n);
  if (k >= np) return;
  const int p = pairs[k].x, q = pairs[k].y;
  if (p >= n || q >= n) return;
  const Rot r = rot[k];
  if (r.s == 0.0) return;
  // e^{-i phi} = (cph, -sph)
  for (int m = 0; m < 2; ++m) {
    z64* X = m == 0 ? A : V;
    if (!X) continue;
    const z64 xp = X[(long long)i * n + p], xq = X[(long long)i * n + q];
    const z64 eq = {xq.x * r.cph + xq.y * r.sph, xq.y * r.cph - xq.x * r.sph};  // xq e^{-i phi}
    X[(long long)i * n + p] = z64{r.c * xp.x - r.s * eq.x, r.c * xp.y - r.s * eq.y};
    X[(long long)i * n + q] = z64{r.s * xp.x + r.c * eq.x, r.s * xp.y + r.c * eq.y};
  }
}

// A <- U^H A on rows (p, q) for every column
__global__ void k_jac_rows(z64* A, int n, const int2* pairs, int np, const Rot* rot) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = int(t / n), j = int(t % n);
  if (k >= np) return;
  const int p = pairs[k].x, q = pairs[k].y;
  if (p >= n || q >= n) return;
  const Rot r = rot[k];
  if (r.s == 0.0) return;
  const z64 ap = A[(long long)p * n + j], aq = A[(long long)q * n + j];
  const z64 eq = {aq.x * r.cph - aq.y * r.sph, aq.y * r.cph + aq.x * r.sph};  // aq e^{+i phi}
  A[(long long)p * n + j] = z64{r.c * ap.x - r.s * eq.x, r.c * ap.y - r.s * eq.y};
  A[(long long)q * n + j] = z64{r.s * ap.x + r.c * eq.x, r.s * ap.y + r.c * eq.y};
}

// partial sums of |A_ij|^2 off the diagonal and on it, one pair per block
__global__ void k_jac_norms(const z64* A, int n, double* out) {
  __shared__ double so[256], sd[256];
  double off = 0.0, dia = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < (long long)n * n;
       t += (long long)gridDim.x * blockDim.x) {
    const z64 v = A[t];
    const double m2 = v.x * v.x + v.y * v.y;
    if (t / n == t % n) dia += m2; else off += m2;
  }
  so[threadIdx.x] = off;
  sd[threadIdx.x] = dia;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = so[0];
    out[2 * blockIdx.x + 1] = sd[0];
  }
}

__global__ void k_set_identity(z64* V, int n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  V[t] = z64{(t / n == t % n) ? 1.0 : 0.0, 0.0};
}

// C = op(A) B for small row-major n x n matrices; op = conjugate transpose if ah
__global__ void k_small_mm(const z64* A, const z64* B, z64* C, int n, int ah) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = int(t / n), j = int(t % n);
  double re = 0.0, im = 0.0;
  for (int k = 0; k < n; ++k) {
    z64 a = ah ? A[(long long)k * n + i] : A[(long long)i * n + k];
    if (ah) a.y = -a.y;
    const z64 b = B[(long long)k * n + j];
    re += a.x * b.x - a.y * b.y;
    im += a.x * b.y + a.y * b.x;
  }
  C[t] = z64{re, im};
}

// columns of V scaled: V[:, j] *= s[j]
__global__ void k_scale_cols(z64* V, int n, const double* s) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const double f = s[t % n];
  V[t].x *= f;
  V[t].y *= f;
}

__global__ void k_diag(const z64* A, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[(long long)i * n + i].x;
}

// dst[:, j] = src[:, perm[j]]
__global__ void k_perm_cols(const z64* src, z64* dst, int n, const int* perm) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = int(t / n), j = int(t % n);
  dst[t] = src[(long long)i * n + perm[j]];
}

inline unsigned nblk(long long n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

// Eigen-decomposition of the Hermitian n x n device matrix A (destroyed).
// w (host) receives the ascending eigenvalues; V (device, optional) the
// eigenvectors as columns in the same order.
void eig_hermitian_device(Budget* b, z64* A, int n, double* w, z64* V, hipStream_t st) {
  if (n <= 0) return;
  const int m = n + (n & 1);        // even number of players (a dummy when n is odd)
  const int np = m / 2;
  std::vector<int2> pairs((size_t)(m - 1) * np);
  std::vector<int> pos(m);
  std::iota(pos.begin(), pos.end(), 0);
  for (int r = 0; r < m - 1; ++r) {
    for (int k = 0; k < np; ++k) {
      int p = pos[k], q = pos[m - 1 - k];
      if (p > q) std::swap(p, q);
      pairs[(size_t)r * np + k] = int2{p, q};
    }
    // rotate every position except the first
    const int last = pos[m - 1];
    for (int k = m - 1; k > 1; --k) pos[k] = pos[k - 1];
    pos[1] = last;
  }
  DevMem d_pairs(b, pairs.size() * sizeof(int2));
  DevMem d_rot(b, (size_t)np * sizeof(Rot));
  DevMem d_V(b, (size_t)n * n * sizeof(z64));
  const int nb_norm = 64;
  DevMem d_norm(b, (size_t)nb_norm * 2 * sizeof(double));
  STH_HIP_CHECK(hipMemcpyAsync(d_pairs.as<void>(), pairs.data(), pairs.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_set_identity, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st,
                     d_V.as<z64>(), n);
  std::vector<double> hn(nb_norm * 2);
  for (int sweep = 0; sweep < 40; ++sweep) {
    hipLaunchKernelGGL(k_jac_norms, dim3(nb_norm), dim3(256), 0, st, A, n, d_norm.as<double>());
    STH_HIP_CHECK(hipMemcpyAsync(hn.data(), d_norm.as<void>(), hn.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
    STH_HIP_CHECK(hipStreamSynchronize(st));
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < nb_norm; ++i) {
      off += hn[2 * i];
      dia += hn[2 * i + 1];
    }
    if (!(off == off) || !(dia == dia)) {
      set_error("eigensolver: non-finite matrix entries");
      throw Error(STH_E_INTERNAL);
    }
    if (off <= 1e-30 * (off + dia) || off == 0.0) break;
    for (int r = 0; r < m - 1; ++r) {
      const int2* pr = d_pairs.as<int2>() + (size_t)r * np;
      hipLaunchKernelGGL(k_jac_params, dim3(nblk(np, 128)), dim3(128), 0, st, A, n, pr, np,
                         d_rot.as<Rot>());
      hipLaunchKernelGGL(k_jac_cols, dim3(nblk((long long)np * n, 256)), dim3(256), 0, st, A,
                         d_V.as<z64>(), n, pr, np, d_rot.as<Rot>());
      hipLaunchKernelGGL(k_jac_rows, dim3(nblk((long long)np * n, 256)), dim3(256), 0, st, A, n,
                         pr, np, d_rot.as<Rot>());
    }
    STH_HIP_CHECK(hipGetLastError());
  }
  DevMem d_w(b, (size_t)n * sizeof(double));
  hipLaunchKernelGGL(k_diag, dim3(nblk(n, 128)), dim3(128), 0, st, A, n, d_w.as<double>());
  std::vector<double> wu(n);
  STH_HIP_CHECK(hipMemcpyAsync(wu.data(), d_w.as<void>(), n * sizeof(double),
                               hipMemcpyDeviceToHost, st));
  STH_HIP_CHECK(hipStreamSynchronize(st));
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return wu[a] < wu[c]; });
  for (int i = 0; i < n; ++i) w[i] = wu[perm[i]];
  if (V) {
    DevMem d_perm(b, (size_t)n * sizeof(int));
    STH_HIP_CHECK(hipMemcpyAsync(d_perm.as<void>(), perm.data(), n * sizeof(int),
                                 hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_perm_cols, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st,
                       d_V.as<z64>(), V, n, d_perm.as<int>());
    STH_HIP_CHECK(hipStreamSynchronize(st));
  }
  STH_HIP_CHECK(hipGetLastError());
}

// C = op(A) B on the device (small dense matrices)
void small_mm_device(const z64* A, const z64* B, z64* C, int n, bool ah, hipStream_t st) {
  hipLaunchKernelGGL(k_small_mm, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st, A, B, C, n,
                     ah ? 1 : 0);
  STH_HIP_CHECK(hipGetLastError());
}

void scale_cols_device(z64* V, int n, const double* s_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_cols, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st, V, n,
                     s_dev);
  STH_HIP_CHECK(hipGetLastError());
}

// Ascending eigenvalues of the real symmetric-definite pencil (sym(M), S), n x n
// host matrices, solved on the device: S = U L U^T, T = U L^{-1/2},
// eigenvalues of T^T sym(M) T.
void gen_eig_device(Budget* b, const std::vector<double>& M, const std::vector<double>& S, int n,
                    double* lam, hipStream_t st) {
  std::vector<z64> hm((size_t)n * n), hs((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      hm[(size_t)i * n + j] = z64{0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]), 0.0};
      hs[(size_t)i * n + j] = z64{0.5 * (S[(size_t)i * n + j] + S[(size_t)j * n + i]), 0.0};
    }
  DevMem dM(b, hm.size() * sizeof(z64)), dS(b, hs.size() * sizeof(z64));
  DevMem dU(b, hs.size() * sizeof(z64)), dT(b, hs.size() * sizeof(z64));
  DevMem ds(b, (size_t)n * sizeof(double));
  STH_HIP_CHECK(hipMemcpyAsync(dM.as<void>(), hm.data(), hm.size() * sizeof(z64),
                               hipMemcpyHostToDevice, st));
  STH_HIP_CHECK(hipMemcpyAsync(dS.as<void>(), hs.data(), hs.size() * sizeof(z64),
                               hipMemcpyHostToDevice, st));
  std::vector<double> ls(n);
  eig_hermitian_device(b, dS.as<z64>(), n, ls.data(), dU.as<z64>(), st);
  if (!(ls[0] > 1e-14 * std::fabs(ls[n - 1]))) {
    set_error("chi0 block: the perturbation overlap matrix S is not positive definite "
              "(smallest eigenvalue %.3e)", ls[0]);
    throw Error(STH_E_INVALID);
  }
  std::vector<double> inv(n);
  for (int i = 0; i < n; ++i) inv[i] = 1.0 / std::sqrt(ls[i]);
  STH_HIP_CHECK(hipMemcpyAsync(ds.as<void>(), inv.data(), n * sizeof(double),
                               hipMemcpyHostToDevice, st));
  scale_cols_device(dU.as<z64>(), n, ds.as<double>(), st);        // T = U L^{-1/2}
  small_mm_device(dM.as<z64>(), dU.as<z64>(), dT.as<z64>(), n, false, st);   // M T
  small_mm_device(dU.as<z64>(), dT.as<z64>(), dS.as<z64>(), n, true, st);    // T^H (M T)
  eig_hermitian_device(b, dS.as<z64>(), n, lam, nullptr, st);
}

}  // namespace sth
