// Dense complex contractions on the matrix cores of gfx950 (FP64 and FP32).
//
// The projector products of the Hamiltonian (V_NL = sum |beta> D <beta|) and of
// the valence projector P_v = sum |v><v| are tall-skinny GEMMs over the sphere
// index: C = W^H P (reduction over npw) and Y += W C (npw output rows).  They
// run on v_mfma_f64_16x16x4f64 (FP64 solves) or v_mfma_f32_16x16x4f32 (the
// inner iterations of mixed-precision solves).  A complex product is mapped
// onto real MFMA by interleaving the reduction index: k' = 2k + t, t = 0 for
// the real part and 1 for the imaginary part; the real A' row is the
// interleaved storage itself and the two real B' operands are (re, im) or
// (im, -re) picked per lane.  CG vectors stay FP64 in memory and are rounded
// to the working precision when they are staged in LDS.
//
// MFMA 16x16x4 lane layout (64 lanes, l = lane), measured on gfx950:
//   A[i][k]: i = l % 16, k = l / 16;  B[k][j]: k = l / 16, j = l % 16;
//   D[i][j], register v: j = l % 16 and
//     i = l / 16 + 4 v      for v_mfma_f64_16x16x4f64,
//     i = 4 (l / 16) + v    for v_mfma_f32_16x16x4f32.
#include <cstdlib>

#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row of lane group kq = l / 16, register v
  __device__ static int row(int kq, int v) { return kq + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int kq, int v) { return 4 * kq + v; }
};

constexpr int GT = 64;      // tile rows and columns
constexpr int GK = 16;      // complex reduction elements per LDS stage
constexpr int GTHR = 256;   // 4 waves, 2 x 2 arrangement of 32 x 32 sub-tiles

template <typename T, typename S>
__device__ inline cpx<T> rnd(const S& v) { return cpx<T>{T(v.x), T(v.y)}; }

// waves per SIMD the register allocation is planned for (FP64: three workgroups
// per CU; FP32: four, the most that stay free of spills)
template <typename T>
constexpr int gemm_wpe() { return sizeof(T) == 8 ? 3 : 4; }

// part[s][c][m] = sum_{k in chunk s} conj(A[m][k]) B_c[k]   (accumulated in T)
// Workgroup tile: 64 rows of A x 32 NY columns of B; the 4 waves sit 2 x 2, each
// holding 32 rows x 16 NY columns (2 x NY MFMA tiles, real and imaginary parts).
// NY = 4 (128 columns) halves the re-reads of A per column of B against NY = 2.
// RE: only the real part, Re conj(A) B = A.x B.x + A.y B.y (imaginary part
// written as 0), half the products: the form of Gamma-point systems, whose
// projections are real.
template <typename T, typename TB, int NY, bool RE = false>
__global__ __launch_bounds__(GTHR) __attribute__((amdgpu_waves_per_eu(NY == 2 ? gemm_wpe<T>() : 2))) void k_gemm_ah_b(const cpx<T>* __restrict__ A, int lda, int M,
                                                    VecSet<const TB> B, const int* slots,
                                                    int ncols, int K, int kchunk, cpx<T>* part) {
  using V4 = typename Mfma<T>::v4;
  constexpr int CT = 32 * NY;             // columns of the workgroup tile
  constexpr int NB = CT * GK / GTHR;      // staged B elements per thread
  __shared__ cpx<T> As[GT][GK + 1];
  __shared__ cpx<T> Bs[CT][GK + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // one K-chunk at a time over the whole chip; within it, the m-tiles that share
  // a block of vectors run on one XCD
  int tx, ty;
  xcd_tile2(false, tx, ty);
  const int s = blockIdx.z;
  const int m0 = tx * GT, n0 = ty * CT;
  const int kbeg = s * kchunk, kend = min(K, kbeg + kchunk);
  V4 accr[2][NY], acci[2][NY];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NY; ++b) accr[a][b] = acci[a][b] = V4{0, 0, 0, 0};
  const TB* brow[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int n = n0 + (tid + i * GTHR) / GK;
    brow[i] = (n < ncols) ? B.base + (long long)slots[n] * B.stride : nullptr;
  }
  const int kq = lane >> 4, r16 = lane & 15;
  // the next K-tile is fetched into registers while the current one is multiplied
  cpx<T> ra[4], rb[NB];
  auto fetch = [&](int kb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + i * GTHR, row = idx / GK, c = idx % GK, k = kb + c;
      const int m = m0 + row;
      ra[i] = (m < M && k < kend) ? A[(long long)m * lda + k] : cpx<T>{0, 0};
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * GTHR, c = idx % GK, k = kb + c;
      rb[i] = (brow[i] && k < kend) ? rnd<T>(brow[i][k]) : cpx<T>{0, 0};
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int kb = kbeg; kb < kend; kb += GK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + i * GTHR;
      As[idx / GK][idx % GK] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int idx = tid + i * GTHR;
      Bs[idx / GK][idx % GK] = rb[i];
    }
    __syncthreads();
    if (kb + GK < kend) fetch(kb + GK);
#pragma unroll
    for (int kk = 0; kk < GK / 2; ++kk) {
      const int c = 2 * kk + (kq >> 1);
      const bool im = kq & 1;
      T a[2], br[NY], bi[NY];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cpx<T> w = As[wm * 32 + t * 16 + r16][c];
        a[t] = im ? w.y : w.x;
      }
#pragma unroll
      for (int t = 0; t < NY; ++t) {
        const cpx<T> z = Bs[wn * 16 * NY + t * 16 + r16][c];
        br[t] = im ? z.y : z.x;
        bi[t] = im ? -z.x : z.y;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y) {
          accr[x][y] = Mfma<T>::op(a[x], br[y], accr[x][y]);
          if constexpr (!RE) acci[x][y] = Mfma<T>::op(a[x], bi[y], acci[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 32 + x * 16 + Mfma<T>::row(kq, v);
        const int n = n0 + wn * 16 * NY + y * 16 + r16;
        if (m < M && n < ncols)
          part[((long long)s * ncols + n) * M + m] =
              cpx<T>{accr[x][y][v], RE ? T(0) : acci[x][y][v]};
      }
}

template <typename T>
__global__ void k_reduce_parts(const cpx<T>* part, int nsplit, int ncols, int M,
                               const double* diag, double sgn, cpx<T>* C, int transpose) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)ncols * M) return;
  const int m = int(i % M);
  double re = 0.0, im = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const cpx<T> v = part[(long long)s * ncols * M + i];
    re += v.x;
    im += v.y;
  }
  const double d = sgn * (diag ? diag[m] : 1.0);
  const cpx<T> o = {T(d * re), T(d * im)};
  if (transpose)
    C[(long long)m * ncols + (i / M)] = o;
  else
    C[i] = o;
}

// Y_c[g] = s0 Y_c[g] + sum_m A[m][g] C[c][m]  (+ optional partial dots with dot_in).
// Workgroup tile: 64 rows g x 32 NY columns; each wave 32 g x 16 NY columns.
// The FP64 register budget for three workgroups per CU measured 55 TFLOP/s
// against 48 with the compiler's two-workgroup default.
// RE: C real (its imaginary part is not read), Y.x += sum A.x C and
// Y.y += sum A.y C: each MFMA k-step covers 4 rows m instead of 2, half the
// products (Gamma-point systems).
template <typename T, int NY, bool RE = false>
__global__ __launch_bounds__(GTHR) __attribute__((amdgpu_waves_per_eu(NY == 2 ? gemm_wpe<T>() : 2))) void k_gemm_a_c(
    const cpx<T>* __restrict__ A, int lda, int M, const cpx<T>* __restrict__ C, VecSet<z64> Y,
    const int* slots, int ncols, int K, double s0, VecSet<const z64> dot_in, double* dots) {
  using V4 = typename Mfma<T>::v4;
  constexpr int CT = 32 * NY;             // columns of the workgroup tile
  constexpr int NC = CT * GK / GTHR;      // staged C elements per thread
  __shared__ cpx<T> Ws[GK][GT + 1];
  __shared__ cpx<T> Cs[CT][GK + 1];
  __shared__ double red[CT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = wave & 1, wn = wave >> 1;
  // the column tiles that share a block of W rows run on one XCD, one after the
  // other, so that block is read from memory once
  int tx, ty;
  xcd_tile2(true, tx, ty);
  const int g0 = tx * GT, n0 = ty * CT;
  const int kq = lane >> 4, r16 = lane & 15;
  V4 accr[2][NY], acci[2][NY];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NY; ++b) accr[a][b] = acci[a][b] = V4{0, 0, 0, 0};
  // the next M-tile of W and C is fetched into registers during the multiply
  cpx<T> rw[4], rc[NC];
  auto fetch = [&](int mb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + i * GTHR;
      const int mr = idx / GT, gc = idx % GT;
      const int m = mb + mr, gg = g0 + gc;
      rw[i] = (m < M && gg < K) ? A[(long long)m * lda + gg] : cpx<T>{0, 0};
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int idx = tid + i * GTHR;
      const int nr = idx / GK, mc = idx % GK;
      const int n = n0 + nr, m = mb + mc;
      rc[i] = (n < ncols && m < M) ? C[(long long)n * M + m] : cpx<T>{0, 0};
    }
  };
  if (M > 0) fetch(0);
  for (int mb = 0; mb < M; mb += GK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = tid + i * GTHR;
      Ws[idx / GT][idx % GT] = rw[i];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int idx = tid + i * GTHR;
      Cs[idx / GK][idx % GK] = rc[i];
    }
    __syncthreads();
    if (mb + GK < M) fetch(mb + GK);
    if constexpr (RE) {
      // MFMA k slot kq holds row m = 4 kk + kq
#pragma unroll
      for (int kk = 0; kk < GK / 4; ++kk) {
        const int mm = 4 * kk + kq;
        T ar[2], ai[2], b[NY];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const cpx<T> w = Ws[mm][wg * 32 + t * 16 + r16];
          ar[t] = w.x;
          ai[t] = w.y;
        }
#pragma unroll
        for (int t = 0; t < NY; ++t) b[t] = Cs[wn * 16 * NY + t * 16 + r16][mm].x;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < NY; ++y) {
            if constexpr (sizeof(T) == 4) {   // transposed tile, as below
              accr[x][y] = Mfma<T>::op(b[y], ar[x], accr[x][y]);
              acci[x][y] = Mfma<T>::op(b[y], ai[x], acci[x][y]);
            } else {
              accr[x][y] = Mfma<T>::op(ar[x], b[y], accr[x][y]);
              acci[x][y] = Mfma<T>::op(ai[x], b[y], acci[x][y]);
            }
          }
      }
      __syncthreads();
      continue;
    }
#pragma unroll
    for (int kk = 0; kk < GK / 2; ++kk) {
      const int mm = 2 * kk + (kq >> 1);
      const bool im = kq & 1;
      T a[2], br[NY], bi[NY];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const cpx<T> w = Ws[mm][wg * 32 + t * 16 + r16];
        a[t] = im ? w.y : w.x;
      }
#pragma unroll
      for (int t = 0; t < NY; ++t) {
        const cpx<T> c = Cs[wn * 16 * NY + t * 16 + r16][mm];
        br[t] = im ? -c.y : c.x;
        bi[t] = im ? c.x : c.y;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < NY; ++y) {
          if constexpr (sizeof(T) == 4) {   // transposed tile: column index in the rows
            accr[x][y] = Mfma<T>::op(br[y], a[x], accr[x][y]);
            acci[x][y] = Mfma<T>::op(bi[y], a[x], acci[x][y]);
          } else {
            accr[x][y] = Mfma<T>::op(a[x], br[y], accr[x][y]);
            acci[x][y] = Mfma<T>::op(a[x], bi[y], acci[x][y]);
          }
        }
    }
    __syncthreads();
  }
  if constexpr (sizeof(T) == 4) {
    // FP32: the tile is held transposed, D[n][g] with n = 4 (l / 16) + v and
    // g = l % 16, so that one store instruction writes 16 consecutive g of each
    // of 4 columns (256 B runs) instead of 16 B pieces 64 B apart
    double dsum[NY][4];
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) dsum[y][v] = 0.0;
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + wn * 16 * NY + y * 16 + 4 * kq + v;
        if (n >= ncols) continue;
        z64* yrow = Y.base + (long long)slots[n] * Y.stride;
        const z64* drow = dots ? dot_in.base + (long long)slots[n] * dot_in.stride : nullptr;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int gg = g0 + wg * 32 + x * 16 + r16;
          if (gg < K) {
            z64 o = {double(accr[x][y][v]), double(acci[x][y][v])};
            if (s0 != 0.0) {
              const z64 yo = yrow[gg];
              o.x += s0 * yo.x;
              o.y += s0 * yo.y;
            }
            yrow[gg] = o;
            if (drow) {
              const z64 d = drow[gg];
              dsum[y][v] += d.x * o.x + d.y * o.y;
            }
          }
        }
      }
    if (!dots) return;
    // sum over the 16 lanes that share a column, then over the two g halves
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) dsum[y][v] += __shfl_xor(dsum[y][v], o);
    if (wg == 1 && r16 == 0) {   // column sums of the wg == 1 half
#pragma unroll
      for (int y = 0; y < NY; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wn * 16 * NY + y * 16 + 4 * kq + v] = dsum[y][v];
    }
    __syncthreads();
    if (wg == 0 && r16 == 0) {
#pragma unroll
      for (int y = 0; y < NY; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = wn * 16 * NY + y * 16 + 4 * kq + v;
          const int n = n0 + c;
          if (n < ncols) dots[(long long)n * gridDim.x + tx] = dsum[y][v] + red[c];
        }
    }
    return;
  }
  double dsum[NY];
#pragma unroll
  for (int y = 0; y < NY; ++y) dsum[y] = 0.0;
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    const int n = n0 + wn * 16 * NY + y * 16 + r16;
    if (n >= ncols) continue;
    z64* yrow = Y.base + (long long)slots[n] * Y.stride;
    const z64* drow = dots ? dot_in.base + (long long)slots[n] * dot_in.stride : nullptr;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gg = g0 + wg * 32 + x * 16 + Mfma<T>::row(kq, v);
        if (gg < K) {
          z64 o = {double(accr[x][y][v]), double(acci[x][y][v])};
          if (s0 != 0.0) {   // s0 == 0 never reads Y (it may be uninitialised)
            const z64 yo = yrow[gg];
            o.x += s0 * yo.x;
            o.y += s0 * yo.y;
          }
          yrow[gg] = o;
          if (drow) {
            const z64 d = drow[gg];
            dsum[y] += d.x * o.x + d.y * o.y;
          }
        }
      }
  }
  if (!dots) return;
  // sum over the 4 lane groups that share a column, then over the two g halves
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    dsum[y] += __shfl_xor(dsum[y], 16);
    dsum[y] += __shfl_xor(dsum[y], 32);
  }
  if (wg == 1 && kq == 0) {
#pragma unroll
    for (int y = 0; y < NY; ++y) red[wn * 16 * NY + y * 16 + r16] = dsum[y];
  }
  __syncthreads();
  if (wg == 0 && kq == 0) {
#pragma unroll
    for (int y = 0; y < NY; ++y) {
      const int c = wn * 16 * NY + y * 16 + r16;
      const int n = n0 + c;
      if (n < ncols) dots[(long long)n * gridDim.x + tx] = dsum[y] + red[c];
    }
  }
}

// Column tile of both GEMMs: 128 columns once there are enough columns to fill
// them (STH_GEMM_NY=2 keeps 64)
int gemm_ny() {
  static const int ny = [] {
    const char* e = std::getenv("STH_GEMM_NY");
    return e ? std::atoi(e) : 4;
  }();
  return ny;
}

template <typename T, bool RE>
void gemm_ah_b(const cpx<T>* A, int lda, int M, VecSet<const z64> B, const int* slots, int ncols,
               int K, int kchunk, cpx<T>* part, hipStream_t st) {
  if (ncols <= 0 || M <= 0) return;
  const int nsplit = (K + kchunk - 1) / kchunk;
  if (gemm_ny() == 4 && ncols >= 256) {
    dim3 grid((M + GT - 1) / GT, (ncols + 127) / 128, nsplit);
    hipLaunchKernelGGL((k_gemm_ah_b<T, z64, 4, RE>), grid, dim3(GTHR), 0, st, A, lda, M, B, slots,
                       ncols, K, kchunk, part);
  } else {
    dim3 grid((M + GT - 1) / GT, (ncols + GT - 1) / GT, nsplit);
    hipLaunchKernelGGL((k_gemm_ah_b<T, z64, 2, RE>), grid, dim3(GTHR), 0, st, A, lda, M, B, slots,
                       ncols, K, kchunk, part);
  }
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void reduce_parts(const cpx<T>* part, int nsplit, int ncols, int M, const double* diag,
                  double sgn, cpx<T>* C, hipStream_t st, bool transpose) {
  const long long n = (long long)ncols * M;
  if (n <= 0) return;
  hipLaunchKernelGGL((k_reduce_parts<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     part, nsplit, ncols, M, diag, sgn, C, transpose ? 1 : 0);
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T, bool RE>
void gemm_a_c(const cpx<T>* A, int lda, int M, const cpx<T>* C, VecSet<z64> Y, const int* slots,
              int ncols, int K, double s0, VecSet<const z64> dot_in, double* dots,
              hipStream_t st) {
  if (ncols <= 0) return;
  if (gemm_ny() == 4 && ncols >= 256) {
    dim3 grid(gemm_a_c_tiles(K), (ncols + 127) / 128);
    hipLaunchKernelGGL((k_gemm_a_c<T, 4, RE>), grid, dim3(GTHR), 0, st, A, lda, M, C, Y, slots,
                       ncols, K, s0, dot_in, dots);
  } else {
    dim3 grid(gemm_a_c_tiles(K), (ncols + GT - 1) / GT);
    hipLaunchKernelGGL((k_gemm_a_c<T, 2, RE>), grid, dim3(GTHR), 0, st, A, lda, M, C, Y, slots,
                       ncols, K, s0, dot_in, dots);
  }
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace

void launch_gemm_ah_b(const z64* A, int lda, int M, VecSet<const z64> B, const int* slots,
                      int ncols, int K, int kchunk, z64* part, hipStream_t st, bool real) {
  if (real)
    gemm_ah_b<double, true>(A, lda, M, B, slots, ncols, K, kchunk, part, st);
  else
    gemm_ah_b<double, false>(A, lda, M, B, slots, ncols, K, kchunk, part, st);
}
void launch_gemm_ah_b(const z32* A, int lda, int M, VecSet<const z64> B, const int* slots,
                      int ncols, int K, int kchunk, z32* part, hipStream_t st, bool real) {
  if (real)
    gemm_ah_b<float, true>(A, lda, M, B, slots, ncols, K, kchunk, part, st);
  else
    gemm_ah_b<float, false>(A, lda, M, B, slots, ncols, K, kchunk, part, st);
}

void launch_reduce_parts(const z64* part, int nsplit, int ncols, int M, const double* diag,
                         double sgn, z64* C, hipStream_t st, bool transpose) {
  reduce_parts<double>(part, nsplit, ncols, M, diag, sgn, C, st, transpose);
}
void launch_reduce_parts(const z32* part, int nsplit, int ncols, int M, const double* diag,
                         double sgn, z32* C, hipStream_t st, bool transpose) {
  reduce_parts<float>(part, nsplit, ncols, M, diag, sgn, C, st, transpose);
}

void launch_gemm_a_c(const z64* A, int lda, int M, const z64* C, VecSet<z64> Y,
                     const int* slots, int ncols, int K, double s0, VecSet<const z64> dot_in,
                     double* dots, hipStream_t st, bool real) {
  if (real)
    gemm_a_c<double, true>(A, lda, M, C, Y, slots, ncols, K, s0, dot_in, dots, st);
  else
    gemm_a_c<double, false>(A, lda, M, C, Y, slots, ncols, K, s0, dot_in, dots, st);
}
void launch_gemm_a_c(const z32* A, int lda, int M, const z32* C, VecSet<z64> Y,
                     const int* slots, int ncols, int K, double s0, VecSet<const z64> dot_in,
                     double* dots, hipStream_t st, bool real) {
  if (real)
    gemm_a_c<float, true>(A, lda, M, C, Y, slots, ncols, K, s0, dot_in, dots, st);
  else
    gemm_a_c<float, false>(A, lda, M, C, Y, slots, ncols, K, s0, dot_in, dots, st);
}

}  // namespace sth
