// Kernels of the batched Lanczos chains (paper, Section 3: the Lanczos vectors
// of the frequency-dependent response, equation "lanczos", one chain per (PDEP
// vector, orbital), each new vector orthogonalised against the previous ones of
// its chain).
//
// Chains are columns: vector (k, m) of the chain store is Q + (k nm + m) npw
// (k = step, m = chain).  Dot products are fixed-order block reductions
// (deterministic), complex, FP64.
#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

constexpr int kDotThreads = 256;

// out[m * ldo + k] = sum_g conj(X[k xs_k + m xs_m + g]) Y[m ys_m + g]
__global__ __launch_bounds__(kDotThreads) void k_chain_dots(const z64* X, long long xs_k,
                                                           long long xs_m, const z64* Y,
                                                           long long ys_m, int n, z64* out,
                                                           int ldo) {
  __shared__ double re[kDotThreads], im[kDotThreads];
  const int k = blockIdx.x, m = blockIdx.y;
  const z64* x = X + k * xs_k + m * xs_m;
  const z64* y = Y + m * ys_m;
  double a = 0.0, b = 0.0;
  for (int g = threadIdx.x; g < n; g += kDotThreads) {
    const z64 u = x[g], v = y[g];
    a += u.x * v.x + u.y * v.y;
    b += u.x * v.y - u.y * v.x;
  }
  re[threadIdx.x] = a;
  im[threadIdx.x] = b;
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      re[threadIdx.x] += re[threadIdx.x + h];
      im[threadIdx.x] += im[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m * ldo + k] = z64{re[0], im[0]};
}

// r_m = Hq_m - alpha_m q_m - beta_m qprev_m   (qprev may be null: the first step)
__global__ void k_lanczos_three_term(const z64* Hq, const z64* q, const z64* qprev,
                                     const z64* alpha, const double* beta, int nm, int n, z64* r) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nm * n) return;
  const int m = int(t / n);
  const double a = alpha[m].x;
  z64 v = Hq[t];
  v.x -= a * q[t].x;
  v.y -= a * q[t].y;
  if (qprev) {
    const double b = beta[m];
    v.x -= b * qprev[t].x;
    v.y -= b * qprev[t].y;
  }
  r[t] = v;
}

// r_m -= sum_{k < l} c[m * ldc + k] Q[(k nm + m) n + g]
__global__ void k_chain_orth(const z64* Q, int nm, int n, const z64* c, int ldc, int l, z64* r) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nm * n) return;
  const int m = int(t / n);
  const int g = int(t - (long long)m * n);
  double ax = 0.0, ay = 0.0;
  for (int k = 0; k < l; ++k) {
    const z64 w = c[m * ldc + k];
    const z64 v = Q[((long long)k * nm + m) * n + g];
    ax += w.x * v.x - w.y * v.y;
    ay += w.x * v.y + w.y * v.x;
  }
  r[t].x -= ax;
  r[t].y -= ay;
}

// out_m = in_m / s[m]
__global__ void k_chain_div(const z64* in, const double* s, int nm, int n, z64* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nm * n) return;
  const double f = 1.0 / s[t / n];
  out[t] = z64{in[t].x * f, in[t].y * f};
}

// out = a A + b B + c C over n complex elements (C may be null); out may alias C
__global__ void k_block_axpbypcz(long long n, double a, const z64* A, double b, const z64* B,
                                 double c, const z64* C, z64* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const z64 x = A[t], y = B[t];
  double re = a * x.x + b * y.x, im = a * x.y + b * y.y;
  if (C) {
    const z64 z = C[t];
    re += c * z.x;
    im += c * z.y;
  }
  out[t] = z64{re, im};
}

inline unsigned nblk(long long n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

void launch_block_axpbypcz(long long n, double a, const z64* A, double b, const z64* B, double c,
                           const z64* C, z64* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_block_axpbypcz, dim3(nblk(n, 256)), dim3(256), 0, st, n, a, A, b, B, c, C,
                     out);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_chain_dots(const z64* X, long long xs_k, long long xs_m, int nk, const z64* Y,
                       long long ys_m, int nm, int n, z64* out, int ldo, hipStream_t st) {
  if (nk <= 0 || nm <= 0) return;
  hipLaunchKernelGGL(k_chain_dots, dim3(nk, nm), dim3(kDotThreads), 0, st, X, xs_k, xs_m, Y,
                     ys_m, n, out, ldo);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_lanczos_three_term(const z64* Hq, const z64* q, const z64* qprev, const z64* alpha,
                               const double* beta, int nm, int n, z64* r, hipStream_t st) {
  const long long tot = (long long)nm * n;
  hipLaunchKernelGGL(k_lanczos_three_term, dim3(nblk(tot, 256)), dim3(256), 0, st, Hq, q, qprev,
                     alpha, beta, nm, n, r);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_chain_orth(const z64* Q, int nm, int n, const z64* c, int ldc, int l, z64* r,
                       hipStream_t st) {
  if (l <= 0) return;
  const long long tot = (long long)nm * n;
  hipLaunchKernelGGL(k_chain_orth, dim3(nblk(tot, 256)), dim3(256), 0, st, Q, nm, n, c, ldc, l,
                     r);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_chain_div(const z64* in, const double* s, int nm, int n, z64* out, hipStream_t st) {
  const long long tot = (long long)nm * n;
  hipLaunchKernelGGL(k_chain_div, dim3(nblk(tot, 256)), dim3(256), 0, st, in, s, nm, n, out);
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
