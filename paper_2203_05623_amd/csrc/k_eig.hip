// Dense Hermitian eigensolvers for the Rayleigh-Ritz problems of the path
// (valence subspaces, dielectric Davidson, chi0 block), FP64 on the device.
//
// Small problems: cyclic two-sided Jacobi with a round-robin (tournament) ordering: every
// round rotates n/2 disjoint index pairs at once, so a round is two fully
// parallel kernels (columns, then rows).  For a pair (p, q) with
// A_pq = |b| e^{i phi}, the unitary U = diag(1, e^{-i phi}) R, R the real
// Jacobi rotation of [[A_pp, |b|], [|b|, A_qq]] (Golub & Van Loan, symmetric
// Schur decomposition), zeroes A_pq in U^H A U.  Eigenvectors accumulate in
// V <- V U.
//
// Larger problems (n > kJacobiMax): Householder reduction to a real symmetric
// tridiagonal matrix on the device, A = Q T Q^H (one reflector per column,
// the phase of each subdiagonal absorbed so that T is real), the implicit QL
// iteration with Wilkinson shifts on T on the host (Bowdler, Martin, Reinsch
// and Wilkinson; Golub & Van Loan, the symmetric tridiagonal QR step), its
// plane rotations replayed on the device on the eigenvector matrix Z (one
// thread per row), and the back-transformation X = Q Z, one reflector at a
// time.  Matrices are row-major n x n complex (z64).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
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

// Cyclic Jacobi: eigen-decomposition of the Hermitian n x n device matrix A
// (destroyed); w (host) ascending eigenvalues, V (device, optional) eigenvectors
// as columns in the same order.
static void eig_hermitian_jacobi(Budget* b, z64* A, int n, double* w, z64* V, hipStream_t st) {
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

// ---------------------------------------------------------------- tridiagonal route
namespace {

constexpr int kJacobiMax = 64;   // Jacobi below this size, the tridiagonal route above

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block-wide sum over 256 threads (every thread gets the result)
__device__ inline double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  const double r = sh[0] + sh[1] + sh[2] + sh[3];
  return r;
}

// Reflector of step k: x = A[k+1.., k] (the conjugate of row k right of the
// diagonal, A Hermitian).  H = I - tau v v^H with v_0 = 1 and H^H x = beta e_0,
// beta real: beta = -sign(Re x_0) |x|, tau = (beta - x_0^*)... written out below.
// Stores v in R[k][0..m), tau[k], d[k] = Re A_kk, e[k] = beta.
__global__ void __launch_bounds__(256) k_hh_reflector(const z64* A, int n, int k, z64* R,
                                                      z64* tau, double* d, double* e) {
  __shared__ double sh[4];
  const int m = n - k - 1;
  const z64* row = A + (long long)k * n + k + 1;
  double part = 0.0;
  for (int j = 1 + threadIdx.x; j < m; j += 256) part += row[j].x * row[j].x + row[j].y * row[j].y;
  const double xn2 = block_sum256(part, sh);
  const z64 a = {row[0].x, -row[0].y};   // x_0 = conj(A[k][k+1])
  z64 t{0.0, 0.0};
  double beta = a.x;
  z64 scale{0.0, 0.0};
  if (xn2 > 0.0 || a.y != 0.0) {
    const double nrm = sqrt(a.x * a.x + a.y * a.y + xn2);
    beta = a.x >= 0.0 ? -nrm : nrm;
    t = z64{(beta - a.x) / beta, -a.y / beta};
    // scale = 1 / (x_0 - beta)
    const double ur = a.x - beta, ui = a.y, den = ur * ur + ui * ui;
    scale = z64{ur / den, -ui / den};
  }
  z64* v = R + (long long)k * n;
  for (int j = threadIdx.x; j < m; j += 256) {
    if (j == 0) {
      v[0] = z64{1.0, 0.0};
    } else {
      const z64 x = {row[j].x, -row[j].y};
      v[j] = z64{x.x * scale.x - x.y * scale.y, x.x * scale.y + x.y * scale.x};
    }
  }
  if (threadIdx.x == 0) {
    tau[k] = t;
    d[k] = A[(long long)k * n + k].x;
    e[k] = beta;
  }
}

// y = A22 v on the trailing block A22 = A[k+1.., k+1..]: one wavefront per row
__global__ void __launch_bounds__(256) k_hh_matvec(const z64* A, int n, int k, const z64* R,
                                                   z64* y) {
  const int m = n - k - 1;
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= m) return;
  const z64* row = A + (long long)(k + 1 + r) * n + k + 1;
  const z64* v = R + (long long)k * n;
  double re = 0.0, im = 0.0;
  for (int c = lane; c < m; c += 64) {
    const z64 a = row[c], b = v[c];
    re += a.x * b.x - a.y * b.y;
    im += a.x * b.y + a.y * b.x;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) y[r] = z64{re, im};
}

// s = Re v^H y, w = tau y - |tau|^2 s v / 2 (one workgroup)
__global__ void __launch_bounds__(256) k_hh_w(int n, int k, const z64* R, const z64* tau,
                                              const z64* y, z64* w) {
  __shared__ double sh[4];
  const int m = n - k - 1;
  const z64* v = R + (long long)k * n;
  double part = 0.0;
  for (int j = threadIdx.x; j < m; j += 256) part += v[j].x * y[j].x + v[j].y * y[j].y;
  const double s = block_sum256(part, sh);
  const z64 t = tau[k];
  const double h = 0.5 * (t.x * t.x + t.y * t.y) * s;
  for (int j = threadIdx.x; j < m; j += 256) {
    const z64 yy = y[j];
    w[j] = z64{t.x * yy.x - t.y * yy.y - h * v[j].x, t.x * yy.y + t.y * yy.x - h * v[j].y};
  }
}

// A22 -= v w^H + w v^H
__global__ void __launch_bounds__(256) k_hh_rank2(z64* A, int n, int k, const z64* R,
                                                  const z64* w) {
  const int m = n - k - 1;
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)m * m) return;
  const int r = int(t / m), c = int(t % m);
  const z64* v = R + (long long)k * n;
  const z64 vr = v[r], wr = w[r], vc = v[c], wc = w[c];
  // v_r conj(w_c) + w_r conj(v_c)
  const double re = vr.x * wc.x + vr.y * wc.y + wr.x * vc.x + wr.y * vc.y;
  const double im = vr.y * wc.x - vr.x * wc.y + wr.y * vc.x - wr.x * vc.y;
  z64& a = A[(long long)(k + 1 + r) * n + k + 1 + c];
  a.x -= re;
  a.y -= im;
}

// Plane rotations of the QL sweeps replayed on Z (real n x n, column i of Z
// contiguous: Zc[i * n + row]), one thread per row.  A sweep rotates the column
// pairs (i, i + 1) for i = top, top - 1, ..., top - count + 1:
//   f = Z_{i+1};  Z_{i+1} = s Z_i + c f;  Z_i = c Z_i - s f.
// Within a sweep the columns read (i) are never those written (i + 1 > i), so
// the loads of a group of eight go out before its arithmetic.
struct Sweep {
  int top, count;
  long long off;
};

__global__ void __launch_bounds__(64) k_ql_rotate(double* Zc, int n, const Sweep* sw, int nsw,
                                                 const double2* cs) {
  const int row = blockIdx.x * 64 + threadIdx.x;
  if (row >= n) return;
  for (int q = 0; q < nsw; ++q) {
    const Sweep S = sw[q];
    const double2* g = cs + S.off;
    double carry = Zc[(long long)(S.top + 1) * n + row];
    int idx = 0;
    for (; idx + 8 <= S.count; idx += 8) {
      double z[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) z[u] = Zc[(long long)(S.top - idx - u) * n + row];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 r = g[idx + u];
        const int i = S.top - idx - u;
        Zc[(long long)(i + 1) * n + row] = r.y * z[u] + r.x * carry;
        carry = r.x * z[u] - r.y * carry;
      }
    }
    for (; idx < S.count; ++idx) {
      const double2 r = g[idx];
      const int i = S.top - idx;
      const double zi = Zc[(long long)i * n + row];
      Zc[(long long)(i + 1) * n + row] = r.y * zi + r.x * carry;
      carry = r.x * zi - r.y * carry;
    }
    Zc[(long long)(S.top - S.count + 1) * n + row] = carry;
  }
}

__global__ void k_set_identity_real(double* Z, int n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  Z[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// V[r][j] = Z[r][perm[j]] (complex, row-major) from Zc
__global__ void k_z_to_v(const double* Zc, int n, const int* perm, z64* V) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int r = int(t / n), j = int(t % n);
  V[t] = z64{Zc[(long long)perm[j] * n + r], 0.0};
}

// rows k+1.. of V: V -= tau v (v^H V); a workgroup owns 32 columns, 8 row groups
__global__ void __launch_bounds__(256) k_hh_apply(z64* V, int n, int k, const z64* R,
                                                  const z64* tau) {
  __shared__ double sre[8][33], sim[8][33];
  const int m = n - k - 1;
  const int cl = threadIdx.x & 31, rg = threadIdx.x >> 5;
  const int c = blockIdx.x * 32 + cl;
  const z64* v = R + (long long)k * n;
  z64* base = V + (long long)(k + 1) * n;
  double re = 0.0, im = 0.0;
  if (c < n)
    for (int r = rg; r < m; r += 8) {
      const z64 a = base[(long long)r * n + c], b = v[r];   // conj(b) a
      re += b.x * a.x + b.y * a.y;
      im += b.x * a.y - b.y * a.x;
    }
  sre[rg][cl] = re;
  sim[rg][cl] = im;
  __syncthreads();
  double ur = 0.0, ui = 0.0;
  for (int q = 0; q < 8; ++q) {
    ur += sre[q][cl];
    ui += sim[q][cl];
  }
  if (c >= n) return;
  const z64 t = tau[k];
  const z64 tu = {t.x * ur - t.y * ui, t.x * ui + t.y * ur};
  for (int r = rg; r < m; r += 8) {
    const z64 b = v[r];
    z64& a = base[(long long)r * n + c];
    a.x -= b.x * tu.x - b.y * tu.y;
    a.y -= b.x * tu.y + b.y * tu.x;
  }
}

// Implicit QL with Wilkinson shifts on the real symmetric tridiagonal matrix
// (diagonal d, subdiagonal e[0..n-2]); d receives the eigenvalues (unordered).
// When `rec` is set, every plane rotation is recorded (sweeps and (c, s)
// pairs) for the eigenvector matrix.
void tridiag_ql(std::vector<double>& d, std::vector<double> e, std::vector<Sweep>* sweeps,
                std::vector<double2>* cs) {
  const int n = int(d.size());
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= std::numeric_limits<double>::epsilon() * dd) break;
      }
      if (m == l) break;
      if (iter == 200) {
        set_error("eigensolver: QL iteration did not converge");
        throw Error(STH_E_INTERNAL);
      }
      // Wilkinson-type shift from the leading 2 x 2 block of the unreduced part
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      Sweep sw{m - 1, 0, cs ? (long long)cs->size() : 0};
      int i = m - 1;
      bool underflow = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {   // the rotation is the identity: the matrix splits here
          d[i + 1] -= p;
          e[m] = 0.0;
          underflow = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        if (cs) cs->push_back(double2{c, s});
        sw.count += 1;
      }
      if (sweeps && sw.count > 0) sweeps->push_back(sw);
      if (underflow) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
}

void eig_hermitian_tridiag(Budget* b, z64* A, int n, double* w, z64* V, hipStream_t st) {
  DevMem dR(b, (size_t)n * n * sizeof(z64)), dtau(b, (size_t)n * sizeof(z64));
  DevMem dd(b, (size_t)n * sizeof(double)), de(b, (size_t)n * sizeof(double));
  DevMem dy(b, (size_t)n * sizeof(z64)), dw(b, (size_t)n * sizeof(z64));
  for (int k = 0; k + 1 < n; ++k) {
    const int m = n - k - 1;
    hipLaunchKernelGGL(k_hh_reflector, dim3(1), dim3(256), 0, st, A, n, k, dR.as<z64>(),
                       dtau.as<z64>(), dd.as<double>(), de.as<double>());
    hipLaunchKernelGGL(k_hh_matvec, dim3(nblk(m, 4)), dim3(256), 0, st, A, n, k, dR.as<z64>(),
                       dy.as<z64>());
    hipLaunchKernelGGL(k_hh_w, dim3(1), dim3(256), 0, st, n, k, dR.as<z64>(), dtau.as<z64>(),
                       dy.as<z64>(), dw.as<z64>());
    hipLaunchKernelGGL(k_hh_rank2, dim3(nblk((long long)m * m, 256)), dim3(256), 0, st, A, n, k,
                       dR.as<z64>(), dw.as<z64>());
  }
  STH_HIP_CHECK(hipGetLastError());
  std::vector<double> d(n), e(n, 0.0);
  z64 last;
  STH_HIP_CHECK(hipMemcpyAsync(&last, A + (long long)(n - 1) * n + n - 1, sizeof(z64),
                               hipMemcpyDeviceToHost, st));
  if (n > 1) {
    STH_HIP_CHECK(hipMemcpyAsync(d.data(), dd.as<void>(), (n - 1) * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
    STH_HIP_CHECK(hipMemcpyAsync(e.data(), de.as<void>(), (n - 1) * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
  }
  STH_HIP_CHECK(hipStreamSynchronize(st));
  d[n - 1] = last.x;
  for (double x : d)
    if (!(x == x)) {
      set_error("eigensolver: non-finite matrix entries");
      throw Error(STH_E_INTERNAL);
    }
  std::vector<Sweep> sweeps;
  std::vector<double2> cs;
  tridiag_ql(d, e, V ? &sweeps : nullptr, V ? &cs : nullptr);
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return d[a] < d[c]; });
  for (int i = 0; i < n; ++i) w[i] = d[perm[i]];
  if (!V) return;
  DevMem dZ(b, (size_t)n * n * sizeof(double));
  DevMem dsw(b, std::max<size_t>(sweeps.size(), 1) * sizeof(Sweep));
  DevMem dcs(b, std::max<size_t>(cs.size(), 1) * sizeof(double2));
  DevMem dperm(b, (size_t)n * sizeof(int));
  hipLaunchKernelGGL(k_set_identity_real, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st,
                     dZ.as<double>(), n);
  if (!sweeps.empty()) {
    STH_HIP_CHECK(hipMemcpyAsync(dsw.as<void>(), sweeps.data(), sweeps.size() * sizeof(Sweep),
                                 hipMemcpyHostToDevice, st));
    STH_HIP_CHECK(hipMemcpyAsync(dcs.as<void>(), cs.data(), cs.size() * sizeof(double2),
                                 hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ql_rotate, dim3(nblk(n, 64)), dim3(64), 0, st, dZ.as<double>(), n,
                       dsw.as<Sweep>(), int(sweeps.size()), dcs.as<double2>());
  }
  STH_HIP_CHECK(hipMemcpyAsync(dperm.as<void>(), perm.data(), n * sizeof(int),
                               hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_z_to_v, dim3(nblk((long long)n * n, 256)), dim3(256), 0, st,
                     dZ.as<double>(), n, dperm.as<int>(), V);
  for (int k = n - 2; k >= 0; --k)
    hipLaunchKernelGGL(k_hh_apply, dim3(nblk(n, 32)), dim3(256), 0, st, V, n, k, dR.as<z64>(),
                       dtau.as<z64>());
  STH_HIP_CHECK(hipGetLastError());
  STH_HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace

// Eigen-decomposition of the Hermitian n x n device matrix A (destroyed).
// w (host) receives the ascending eigenvalues; V (device, optional) the
// eigenvectors as columns in the same order.  The environment variable
// STH_EIG=jacobi or tridiag forces one route.
void eig_hermitian_device(Budget* b, z64* A, int n, double* w, z64* V, hipStream_t st) {
  if (n <= 0) return;
  const char* ev = std::getenv("STH_EIG");
  const bool jac = ev && std::strcmp(ev, "jacobi") == 0   ? true
                   : ev && std::strcmp(ev, "tridiag") == 0 ? false
                                                           : n <= kJacobiMax;
  if (jac)
    eig_hermitian_jacobi(b, A, n, w, V, st);
  else
    eig_hermitian_tridiag(b, A, n, w, V, st);
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
