// Half-sphere forms of the projector products for systems whose vectors are
// real in real space (Gamma-point sampling, paper Section 3): then every
// coefficient vector satisfies c(-G) = conj c(G), the projections
// C = W^H x are real, and
//   C = 2 Re sum_{G in H} conj(W(G)) x(G) - Re(conj(W(0)) x(0)),
// with H the half of the sphere that follows G = 0 in the internal (stick-major)
// order, G = 0 included; Y += W C needs only the half H, the rest is
// Y(-G) = conj Y(G).  The GEMM kernels run on the half through pointer
// offsets, the FP64 / FP32 ones as real products (only Re conj(W) x, and C
// taken as real); these kernels do the reduction with the G = 0 correction,
// the mirror copy and the <a, b> tile partials over the whole sphere.
#include <algorithm>

#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

// C[c][m] = sgn d_m (2 Re sum_s part[s][c][m] - Re(conj(W[m][k0]) x_c[k0])
//                    - 2 Re sum_{kh <= k < k0} conj(W[m][k]) x_c[k]), real
template <typename T, typename TW>
__global__ void k_reduce_parts_gamma(const cpx<T>* part, int nsplit, int ncols, int M,
                                     const double* diag, double sgn, cpx<T>* C, const TW* W,
                                     int ldw, int k0, int kh, VecSet<const z64> X,
                                     const int* slots) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)ncols * M) return;
  const int c = int(i / M), m = int(i - (long long)c * M);
  double re = 0.0;
  for (int s = 0; s < nsplit; ++s) re += part[(long long)s * ncols * M + i].x;
  const TW* w = W + (long long)m * ldw;
  const z64* x = X.base + (long long)slots[c] * X.stride;
  double extra = 0.0;
  for (int k = kh; k < k0; ++k) extra += double(w[k].x) * x[k].x + double(w[k].y) * x[k].y;
  const double g0 = double(w[k0].x) * x[k0].x + double(w[k0].y) * x[k0].y;
  const double d = sgn * (diag ? diag[m] : 1.0);
  C[i] = cpx<T>{T(d * (2.0 * (re - extra) - g0)), T(0)};
}

// Y[mirror[i]] = conj(Y[k0 + 1 + i]) and Im Y[k0] = 0 for every listed vector:
// the projection onto vectors that are real in real space.  The half-sphere
// products never see Im Y(0) (nor the antisymmetric part), so one left by the
// FFT's rounding would meet an operator that is not Hermitian and grow over
// the iterations.
__global__ void k_mirror(VecSet<z64> Y, const int* slots, int k0, int nmir, const int* mirror) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  z64* y = Y.base + (long long)slots[blockIdx.y] * Y.stride;
  if (i == 0) y[k0].y = 0.0;
  if (i >= nmir) return;
  const z64 v = y[k0 + 1 + i];
  y[mirror[i]] = z64{v.x, -v.y};
}

// dots[c][t] = sum_{g in [64 t, 64 t + 64)} Re(conj(a_g) b_g), the tile layout of
// the Y += W C epilogue, over the whole sphere (fixed summation order)
__global__ __launch_bounds__(64) void k_dots_tiles(VecSet<const z64> a, VecSet<const z64> b,
                                                  const int* slots, int npw, int ntile,
                                                  double* dots) {
  const int c = blockIdx.y, t = blockIdx.x, g = t * 64 + threadIdx.x;
  double v = 0.0;
  if (g < npw) {
    const z64 x = a.base[(long long)slots[c] * a.stride + g];
    const z64 y = b.base[(long long)slots[c] * b.stride + g];
    v = x.x * y.x + x.y * y.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (threadIdx.x == 0) dots[(long long)c * ntile + t] = v;
}

// out[r] = max(max_k |W[r][mirror k] - conj W[r][k0 + 1 + k]|, |Im W[r][k0]|),
// out[R + r] = max_k |W[r][k]|
template <typename TW>
__global__ __launch_bounds__(256) void k_sym_check(const TW* W, int R, int npw, int k0, int nmir,
                                                   const int* mirror, double* out) {
  const int r = blockIdx.x;
  const TW* w = W + (long long)r * npw;
  double dev = threadIdx.x == 0 ? fabs(double(w[k0].y)) : 0.0, mag = 0.0;
  for (int i = threadIdx.x; i < nmir; i += 256) {
    const TW a = w[k0 + 1 + i], b = w[mirror[i]];
    dev = fmax(dev, fabs(double(a.x) - double(b.x)) + fabs(double(a.y) + double(b.y)));
  }
  for (int k = threadIdx.x; k < npw; k += 256) mag = fmax(mag, fabs(double(w[k].x)) + fabs(double(w[k].y)));
  __shared__ double sd[256], sm[256];
  sd[threadIdx.x] = dev;
  sm[threadIdx.x] = mag;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + o]);
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[r] = sd[0];
    out[R + r] = sm[0];
  }
}

}  // namespace

template <typename T, typename TW>
void launch_reduce_parts_gamma(const cpx<T>* part, int nsplit, int ncols, int M,
                               const double* diag, double sgn, cpx<T>* C, const TW* W, int ldw,
                               int k0, int kh, VecSet<const z64> X, const int* slots,
                               hipStream_t st) {
  const long long n = (long long)ncols * M;
  if (n <= 0) return;
  if (kh > k0 || kh < 0) {
    set_error("gamma reduction: half start %d after G = 0 at %d", kh, k0);
    throw Error(STH_E_INTERNAL);
  }
  hipLaunchKernelGGL((k_reduce_parts_gamma<T, TW>), dim3((unsigned)((n + 255) / 256)), dim3(256),
                     0, st, part, nsplit, ncols, M, diag, sgn, C, W, ldw, k0, kh, X, slots);
  STH_HIP_CHECK(hipGetLastError());
}
template void launch_reduce_parts_gamma<double, z64>(const z64*, int, int, int, const double*,
                                                     double, z64*, const z64*, int, int, int,
                                                     VecSet<const z64>, const int*, hipStream_t);
template void launch_reduce_parts_gamma<float, z32>(const z32*, int, int, int, const double*,
                                                    double, z32*, const z32*, int, int, int,
                                                    VecSet<const z64>, const int*, hipStream_t);

void launch_mirror(VecSet<z64> Y, const int* slots, int ncols, int k0, int nmir,
                   const int* mirror, hipStream_t st) {
  if (ncols <= 0) return;
  const unsigned nb = (unsigned)std::max(1, (nmir + 255) / 256);
  hipLaunchKernelGGL(k_mirror, dim3(nb, (unsigned)ncols), dim3(256), 0, st, Y, slots, k0, nmir,
                     mirror);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_dots_tiles(VecSet<const z64> a, VecSet<const z64> b, const int* slots, int ncols,
                       int npw, int ntile, double* dots, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_dots_tiles, dim3((unsigned)ntile, (unsigned)ncols), dim3(64), 0, st, a, b,
                     slots, npw, ntile, dots);
  STH_HIP_CHECK(hipGetLastError());
}

void launch_sym_check(const z64* W, int R, int npw, int k0, int nmir, const int* mirror,
                      double* out, hipStream_t st) {
  if (R <= 0) return;
  hipLaunchKernelGGL(k_sym_check<z64>, dim3((unsigned)R), dim3(256), 0, st, W, R, npw, k0, nmir,
                     mirror, out);
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
