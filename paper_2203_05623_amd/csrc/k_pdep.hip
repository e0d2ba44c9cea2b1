// Kernels of the dielectric eigensolver (paper, Section 3: the response is
// represented by eigenpairs of v^{1/2} chi0 v^{1/2}, found by a Davidson
// iteration that applies chi0 through the Sternheimer solves).
//
// Trial vectors are real functions on the full N^3 grid, band-limited to the
// density sphere.  v^{1/2} acts in reciprocal space: a full-grid forward FFT
// (planes along i2 and i1, then lines along i0), a multiply by
// sqrt(4 pi) / |G| inside the density sphere (zero at G = 0 and outside), and
// the inverse FFT.  The Rayleigh-Ritz products are real dot products over the
// grid with the weight Omega / N^3 (fixed-order block reductions).
#include <algorithm>
#include <cmath>

#include "errors.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

template <int N, int P>
constexpr int grid_fft_threads() {
  const int t = RadixPlan<N, P>::threads(N);
  return t < 256 ? 256 : t;
}
template <int N>
constexpr size_t grid_fft_lds() {
  return size_t(N) * (N + 1) * sizeof(z64) + N * sizeof(z64);
}

// 2D transform of plane i0 = blockIdx.x of grid blockIdx.y: along i2, then i1
template <int N, int P, int SIGN>
__global__ __launch_bounds__((grid_fft_threads<N, P>())) void k_grid_planes(z64* data,
                                                                          long long stride,
                                                                          const z64* twg) {
  constexpr int NT = grid_fft_threads<N, P>();
  constexpr int NP = N + 1;
  extern __shared__ unsigned char smem_raw[];
  z64* tile = reinterpret_cast<z64*>(smem_raw);
  z64* tw = tile + N * NP;
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  z64* base = data + blockIdx.y * stride + (long long)blockIdx.x * N * N;
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int r = e / N;
    tile[r * NP + (e - r * N)] = base[e];
  }
  __syncthreads();
  RadixPlan<N, P>::template fft<double, SIGN, NT, N>::run(
      tile, N, 1, [](int f) { return f * NP; }, tw);
  RadixPlan<N, P>::template fft<double, SIGN, NT, N>::run(
      tile, N, NP, [](int f) { return f; }, tw);
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int r = e / N;
    base[e] = tile[r * NP + (e - r * N)];
  }
}

// transform along i0 of the lines (i1 = blockIdx.x, every i2) of grid blockIdx.y;
// the slab is read as runs of N consecutive i2 and held as [i2][i0]
template <int N, int P, int SIGN>
__global__ __launch_bounds__((grid_fft_threads<N, P>())) void k_grid_axis0(z64* data,
                                                                         long long stride,
                                                                         const z64* twg) {
  constexpr int NT = grid_fft_threads<N, P>();
  constexpr int NP = N + 1;
  extern __shared__ unsigned char smem_raw[];
  z64* tile = reinterpret_cast<z64*>(smem_raw);
  z64* tw = tile + N * NP;
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  z64* base = data + blockIdx.y * stride + (long long)blockIdx.x * N;
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int i0 = e / N, i2 = e - i0 * N;
    tile[i2 * NP + i0] = base[(long long)i0 * N * N + i2];
  }
  __syncthreads();
  RadixPlan<N, P>::template fft<double, SIGN, NT, N>::run(
      tile, N, 1, [](int f) { return f * NP; }, tw);
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int i0 = e / N, i2 = e - i0 * N;
    base[(long long)i0 * N * N + i2] = tile[i2 * NP + i0];
  }
}

__device__ inline int miller_of(int i, int N) { return 2 * i < N ? i : i - N; }

// Fourier coefficients of grid blockIdx.y scaled by `scale` (sqrt(4 pi) / |G|)^power
// inside the density sphere 0 < |m|^2 <= m2max, zeroed elsewhere
__global__ void k_coulomb_filter(z64* data, long long stride, int N, int m2max, double b,
                                 int power, double scale) {
  const long long n3 = (long long)N * N * N;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  const int i0 = int(t / ((long long)N * N));
  const int rem = int(t - (long long)i0 * N * N);
  const int i1 = rem / N, i2 = rem - (rem / N) * N;
  const int m0 = miller_of(i0, N), m1 = miller_of(i1, N), m2 = miller_of(i2, N);
  const int q = m0 * m0 + m1 * m1 + m2 * m2;
  double f = 0.0;
  if (q > 0 && q <= m2max)
    f = power ? scale * 3.5449077018110320546 / (b * sqrt(double(q))) : scale;  // sqrt(4 pi)
  z64* p = data + blockIdx.y * stride + t;
  const z64 v = *p;
  *p = z64{v.x * f, v.y * f};
}

__global__ void k_real_to_z(const double* in, long long istride, z64* out, long long ostride,
                            long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[blockIdx.y * ostride + t] = z64{in[blockIdx.y * istride + t], 0.0};
}

__global__ void k_z_to_real(const z64* in, long long istride, double* out, long long ostride,
                            long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[blockIdx.y * ostride + t] = in[blockIdx.y * istride + t].x;
}

// C[i][j] = w sum_r A_i[r] B_j[r] for block (i, j): strided partial sums, then a
// fixed-order tree (deterministic)
constexpr int kGramThreads = 256;
__global__ __launch_bounds__(kGramThreads) void k_gram(const double* A, long long lda,
                                                       const double* B, long long ldb, int nb,
                                                       long long n, double w, double* C) {
  __shared__ double red[kGramThreads];
  const double* a = A + blockIdx.x * lda;
  const double* bb = B + blockIdx.y * ldb;
  double s = 0.0;
  for (long long t = threadIdx.x; t < n; t += kGramThreads) s += a[t] * bb[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kGramThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) C[blockIdx.x * nb + blockIdx.y] = w * red[0];
}

// Y_j = beta Y_j + sum_i X_i C[i][j]   (j = blockIdx.y; Y must not alias X)
__global__ void k_combine(const double* X, long long ldx, int m, const double* C, int k,
                          long long n, double beta, double* Y, long long ldy) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int j = blockIdx.y;
  double acc = 0.0;
  for (int i = 0; i < m; ++i) acc += X[i * ldx + t] * C[i * k + j];
  double* y = Y + j * ldy + t;
  *y = (beta != 0.0 ? beta * *y : 0.0) + acc;
}

// R_j = AY_j - lam_j Y_j
__global__ void k_ritz_resid(const double* AY, const double* Y, long long ld, const double* lam,
                             long long n, double* R) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int j = blockIdx.y;
  R[j * ld + t] = AY[j * ld + t] - lam[j] * Y[j * ld + t];
}

__global__ void k_scale_vec(double* x, long long n, double s) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] *= s;
}

inline unsigned nblk(long long n, int b) { return unsigned((n + b - 1) / b); }

template <auto K>
void set_smem_once(size_t bytes) {
  static bool done = false;
  if (!done) {
    STH_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(K),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
  }
}

}  // namespace

#define STH_GRID_DISPATCH(Nval, Pval, ...)                                            \
  do {                                                                                \
    switch ((Nval) * 4 + (Pval)) {                                                    \
      case 24 * 4 + 0: { constexpr int NN = 24, PP = 0; __VA_ARGS__; } break;        \
      case 24 * 4 + 1: { constexpr int NN = 24, PP = 1; __VA_ARGS__; } break;        \
      case 48 * 4 + 0: { constexpr int NN = 48, PP = 0; __VA_ARGS__; } break;        \
      case 48 * 4 + 1: { constexpr int NN = 48, PP = 1; __VA_ARGS__; } break;        \
      case 72 * 4 + 0: { constexpr int NN = 72, PP = 0; __VA_ARGS__; } break;        \
      case 72 * 4 + 1: { constexpr int NN = 72, PP = 1; __VA_ARGS__; } break;        \
      case 96 * 4 + 0: { constexpr int NN = 96, PP = 0; __VA_ARGS__; } break;        \
      case 96 * 4 + 1: { constexpr int NN = 96, PP = 1; __VA_ARGS__; } break;        \
      default:                                                                        \
        set_error("full-grid FFT: unsupported grid %d / plan %d (grids 24..96)", (Nval), \
                  (Pval));                                                            \
        throw Error(STH_E_INVALID);                                                   \
    }                                                                                 \
  } while (0)

void prepare_grid_fft(int N) {
  for (int p = 0; p < kRadixPlansHost; ++p) {
    STH_GRID_DISPATCH(N, p, {
      set_smem_once<k_grid_planes<NN, PP, +1>>(grid_fft_lds<NN>());
      set_smem_once<k_grid_planes<NN, PP, -1>>(grid_fft_lds<NN>());
      set_smem_once<k_grid_axis0<NN, PP, +1>>(grid_fft_lds<NN>());
      set_smem_once<k_grid_axis0<NN, PP, -1>>(grid_fft_lds<NN>());
    });
  }
}

void launch_grid_fft(int N, int plan, int sign, z64* data, long long stride, int ncols,
                     const z64* tw, hipStream_t st) {
  if (ncols <= 0) return;
  if (sign != 1 && sign != -1) {
    set_error("internal: full-grid FFT sign must be +1 or -1");
    throw Error(STH_E_INTERNAL);
  }
  STH_GRID_DISPATCH(N, plan, {
    constexpr size_t sm = grid_fft_lds<NN>();
    const dim3 grid(NN, ncols), blk(grid_fft_threads<NN, PP>());
    if (sign > 0) {
      hipLaunchKernelGGL((k_grid_planes<NN, PP, +1>), grid, blk, sm, st, data, stride, tw);
      hipLaunchKernelGGL((k_grid_axis0<NN, PP, +1>), grid, blk, sm, st, data, stride, tw);
    } else {
      hipLaunchKernelGGL((k_grid_planes<NN, PP, -1>), grid, blk, sm, st, data, stride, tw);
      hipLaunchKernelGGL((k_grid_axis0<NN, PP, -1>), grid, blk, sm, st, data, stride, tw);
    }
  });
  STH_HIP_CHECK(hipGetLastError());
}

void launch_coulomb_filter(z64* data, long long stride, int ncols, int N, int m2max, double b,
                           int power, double scale, hipStream_t st) {
  if (ncols <= 0) return;
  const long long n3 = (long long)N * N * N;
  hipLaunchKernelGGL(k_coulomb_filter, dim3(nblk(n3, 256), ncols), dim3(256), 0, st, data,
                     stride, N, m2max, b, power, scale);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_real_to_z(const double* in, long long istride, z64* out, long long ostride,
                      long long n, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_real_to_z, dim3(nblk(n, 256), ncols), dim3(256), 0, st, in, istride,
                     out, ostride, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_z_to_real(const z64* in, long long istride, double* out, long long ostride,
                      long long n, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_z_to_real, dim3(nblk(n, 256), ncols), dim3(256), 0, st, in, istride,
                     out, ostride, n);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_gram(const double* A, long long lda, int na, const double* B, long long ldb, int nb,
                 long long n, double w, double* C, hipStream_t st) {
  if (na <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_gram, dim3(na, nb), dim3(kGramThreads), 0, st, A, lda, B, ldb, nb, n, w,
                     C);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_combine(const double* X, long long ldx, int m, const double* C, int k, long long n,
                    double beta, double* Y, long long ldy, hipStream_t st) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_combine, dim3(nblk(n, 256), k), dim3(256), 0, st, X, ldx, m, C, k, n,
                     beta, Y, ldy);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_ritz_resid(const double* AY, const double* Y, long long ld, const double* lam, int k,
                       long long n, double* R, hipStream_t st) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_ritz_resid, dim3(nblk(n, 256), k), dim3(256), 0, st, AY, Y, ld, lam, n,
                     R);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_scale_vec(double* x, long long n, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_vec, dim3(nblk(n, 256)), dim3(256), 0, st, x, n, s);
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
