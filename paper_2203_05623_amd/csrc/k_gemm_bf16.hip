// Projector GEMMs of the mixed-precision inner operator on BF16 matrix cores.
//
// Each FP32 operand x is split into x_hi = bf16(x) and x_lo = bf16(x - x_hi)
// (16 significant bits together) and a product is taken as
// a_lo b_hi + a_hi b_lo + a_hi b_hi on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation; the dropped a_lo b_lo term is below 2^-16 relative.  W is split
// once per system (two bf16 planes, rows padded to bf16_ldw(K) complex, so that
// 16-B loads stay aligned and every tile and LDS stage stays inside a row);
// the CG vectors (FP64 in memory) and the small FP32 coefficient block C are
// split while they are staged in LDS.  The complex product uses the same
// interleaved reduction index as the FP64/FP32 kernels: k' = 2k + t, t = 0 for
// the real part, 1 for the imaginary part.
//
// v_mfma_f32_16x16x32_bf16 lane layout (64 lanes, l = lane), measured on gfx950:
//   A[i][k]: i = l % 16, k = 8 (l / 16) + e (e < 8 bf16 values per lane);
//   B[k][j]: k = 8 (l / 16) + e, j = l % 16;  D[i][j], register v: i = 4 (l / 16) + v, j = l % 16.
#include <algorithm>
#include <cstdlib>

#include "errors.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BT = 64;        // tile rows and columns
constexpr int BK = 32;        // complex reduction elements per LDS stage (two MFMA k-steps)
constexpr int BKP = BK + 4;   // LDS row pitch in complex (144 B: 16-B aligned, bank-spread)
constexpr int BTHR = 256;     // 4 waves, 2 x 2 arrangement of 32 x 32 sub-tiles

__device__ inline f4 mfma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// hi / lo parts of a complex FP32 value
__device__ inline void split(float re, float im, bz& hi, bz& lo) {
  hi.x = __bf16(re);
  hi.y = __bf16(im);
  lo.x = __bf16(re - float(hi.x));
  lo.y = __bf16(im - float(hi.y));
}

__device__ inline bf8 ld8(const bz* p) { return *reinterpret_cast<const bf8*>(p); }

// (x0, y0, x1, y1, ...) -> (y0, -x0, y1, -x1, ...)
__device__ inline bf8 swap_neg_odd(bf8 v) {
  bf8 w = __builtin_shufflevector(v, v, 1, 0, 3, 2, 5, 4, 7, 6);
#pragma unroll
  for (int e = 1; e < 8; e += 2) w[e] = -w[e];
  return w;
}
// (x0, y0, ...) -> (x0, -y0, ...)
__device__ inline bf8 neg_odd(bf8 v) {
#pragma unroll
  for (int e = 1; e < 8; e += 2) v[e] = -v[e];
  return v;
}
// (x0, y0, ...) -> (y0, x0, ...)
__device__ inline bf8 swap(bf8 v) { return __builtin_shufflevector(v, v, 1, 0, 3, 2, 5, 4, 7, 6); }

// three-product accumulation of one 16 x 16 tile
__device__ inline f4 acc3(bf8 a_hi, bf8 a_lo, bf8 b_hi, bf8 b_lo, f4 c) {
  c = mfma(a_lo, b_hi, c);
  c = mfma(a_hi, b_lo, c);
  return mfma(a_hi, b_hi, c);
}

// part[s][c][m] = sum_{k in chunk s} conj(W[m][k]) B_c[k]
// Workgroup tile: 32 XT rows of W x 32 YT vectors; the 4 waves sit 2 x 2, each
// holding 16 XT rows x 16 YT vectors (XT x YT MFMA tiles, real and imaginary
// parts).  Both operands come as bf16 hi/lo planes with rows padded to ldw:
// W split once per system, the vectors split once per product by
// k_split_cols (instead of once per row tile of every workgroup, whose FP64
// loads and conversions kept the vector ALU busier than the matrix cores), so
// staging is 16-byte copies.  A 4-complex chunk lies wholly inside or outside
// [kbeg, kend) (both multiples of 4), and chunks of B past kend are zeroed.
template <int XT, int YT>
__global__ __launch_bounds__(BTHR) __attribute__((amdgpu_waves_per_eu(XT * YT > 4 ? 1 : 3))) void k_gemm_ah_b_bf16(
    const bz* __restrict__ Wb, long long wplane, int ldw, int M, const bz* __restrict__ Pb,
    long long pplane, int ncols, int K, int kchunk, z32* part) {
  constexpr int TM = 32 * XT, TN = 32 * YT;
  constexpr int NWC = TM * BK * 2 / 4 / BTHR;   // 16-B chunks of W per thread per stage
  constexpr int NPC = TN * BK * 2 / 4 / BTHR;   // 16-B chunks of the vectors
  constexpr int WPP = TM * (BK / 4);            // chunks per plane
  constexpr int PPP = TN * (BK / 4);
  __shared__ bz As[2][TM][BKP];
  __shared__ bz Bs[2][TN][BKP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // one K-chunk at a time over the whole chip; within it, the m-tiles that share
  // a block of vectors run on one XCD
  int tx, ty;
  xcd_tile2(false, tx, ty);
  const int s = blockIdx.z;
  const int m0 = tx * TM, n0 = ty * TN;
  const int kbeg = s * kchunk, kend = min(K, kbeg + kchunk);
  const int kq = lane >> 4, r16 = lane & 15;
  f4 accr[XT][YT], acci[XT][YT];
#pragma unroll
  for (int a = 0; a < XT; ++a)
#pragma unroll
    for (int b = 0; b < YT; ++b) accr[a][b] = acci[a][b] = f4{0, 0, 0, 0};
  uint4 rw[NWC], rb[NPC];
  auto fetch = [&](int kb) {
#pragma unroll
    for (int i = 0; i < NWC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / WPP, rem = c - pl * WPP, row = rem >> 3, k4 = (rem & 7) * 4;
      const int m = m0 + row;
      const bz* src = Wb + pl * wplane + (long long)m * ldw + kb + k4;
      rw[i] = (m < M) ? *reinterpret_cast<const uint4*>(src) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / PPP, rem = c - pl * PPP, col = rem >> 3, k4 = (rem & 7) * 4;
      const int n = n0 + col;
      const bz* src = Pb + pl * pplane + (long long)n * ldw + kb + k4;
      rb[i] = (n < ncols && kb + k4 < kend) ? *reinterpret_cast<const uint4*>(src)
                                             : uint4{0, 0, 0, 0};
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int kb = kbeg; kb < kend; kb += BK) {
#pragma unroll
    for (int i = 0; i < NWC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / WPP, rem = c - pl * WPP, row = rem >> 3, k4 = (rem & 7) * 4;
      *reinterpret_cast<uint4*>(&As[pl][row][k4]) = rw[i];
    }
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / PPP, rem = c - pl * PPP, col = rem >> 3, k4 = (rem & 7) * 4;
      *reinterpret_cast<uint4*>(&Bs[pl][col][k4]) = rb[i];
    }
    __syncthreads();
    if (kb + BK < kend) fetch(kb + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int k0 = ks * 16 + 4 * kq;
      bf8 bh[YT], bl[YT], bhs[YT], bls[YT];
#pragma unroll
      for (int t = 0; t < YT; ++t) {
        bh[t] = ld8(&Bs[0][wn * 16 * YT + t * 16 + r16][k0]);
        bl[t] = ld8(&Bs[1][wn * 16 * YT + t * 16 + r16][k0]);
        bhs[t] = swap_neg_odd(bh[t]);
        bls[t] = swap_neg_odd(bl[t]);
      }
#pragma unroll
      for (int x = 0; x < XT; ++x) {
        const bf8 ah = ld8(&As[0][wm * 16 * XT + x * 16 + r16][k0]);
        const bf8 al = ld8(&As[1][wm * 16 * XT + x * 16 + r16][k0]);
#pragma unroll
        for (int y = 0; y < YT; ++y) {
          // Re = sum W.x P.x + W.y P.y;  Im = sum W.x P.y - W.y P.x
          accr[x][y] = acc3(ah, al, bh[y], bl[y], accr[x][y]);
          acci[x][y] = acc3(ah, al, bhs[y], bls[y], acci[x][y]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < XT; ++x)
#pragma unroll
    for (int y = 0; y < YT; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 16 * XT + x * 16 + 4 * kq + v;
        const int n = n0 + wn * 16 * YT + y * 16 + r16;
        if (m < M && n < ncols)
          part[((long long)s * ncols + n) * M + m] = z32{accr[x][y][v], acci[x][y][v]};
      }
}

// Y_c[g] = s0 Y_c[g] + sum_m W[m][g] C[c][m]  (+ optional partial dots with dot_in)
// Workgroup tile: 64 rows g x 32 YT columns (each wave 32 g x 16 YT columns);
// YT = 4 reads W once per 128 columns instead of once per 64.
// C comes split as bf16 hi/lo planes Cb[plane][column][Mp] (k_split_c, rows
// zero-padded to Mp, a multiple of BK), staged by 16-byte copies.
template <int YT>
__global__ __launch_bounds__(BTHR) __attribute__((amdgpu_waves_per_eu(YT > 2 ? 2 : 3))) void k_gemm_a_c_bf16(
    const bz* __restrict__ Wb, long long wplane, int ldw, int M, const bz* __restrict__ Cb,
    int Mp, VecSet<z64> Y, const int* slots, int ncols, int K, double s0,
    VecSet<const z64> dot_in, double* dots) {
  constexpr int TN = 32 * YT;
  constexpr int NCC = TN * BK * 2 / 4 / BTHR;   // 16-B chunks of C per thread per stage
  constexpr int CPP = TN * (BK / 4);             // chunks per plane
  const long long cplane = (long long)ncols * Mp;
  __shared__ bz As[2][BT][BKP];   // [plane][g][m]: W staged transposed
  __shared__ bz Cs[2][TN][BKP];   // [plane][column][m]
  __shared__ double red[YT][32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = wave & 1, wn = wave >> 1;
  // the column tiles that share a block of W rows run on one XCD, one after the
  // other, so that block is read from memory once
  int tx, ty;
  xcd_tile2(true, tx, ty);
  const int g0 = tx * BT, n0 = ty * TN;
  const int kq = lane >> 4, r16 = lane & 15;
  f4 accr[2][YT], acci[2][YT];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < YT; ++b) accr[a][b] = acci[a][b] = f4{0, 0, 0, 0};
  // staging: W rows m (both planes) as 16-B chunks of 4 consecutive g, 4 per
  // thread, written transposed; C as 16-B chunks of 4 consecutive m
  uint4 rw[4], rc[NCC];
  auto fetch = [&](int mb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c >> 9, mm = (c & 511) >> 4, g4 = (c & 15) * 4;
      const int m = mb + mm;
      const bz* src = Wb + pl * wplane + (long long)m * ldw + g0 + g4;
      rw[i] = (m < M) ? *reinterpret_cast<const uint4*>(src) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < NCC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / CPP, rem = c - pl * CPP, col = rem >> 3, m4 = (rem & 7) * 4;
      const int n = n0 + col;
      const bz* src = Cb + pl * cplane + (long long)n * Mp + mb + m4;
      rc[i] = (n < ncols) ? *reinterpret_cast<const uint4*>(src) : uint4{0, 0, 0, 0};
    }
  };
  if (M > 0) fetch(0);
  for (int mb = 0; mb < M; mb += BK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c >> 9, mm = (c & 511) >> 4, g4 = (c & 15) * 4;
      const bz* q = reinterpret_cast<const bz*>(&rw[i]);
#pragma unroll
      for (int u = 0; u < 4; ++u) As[pl][g4 + u][mm] = q[u];
    }
#pragma unroll
    for (int i = 0; i < NCC; ++i) {
      const int c = tid + i * BTHR;
      const int pl = c / CPP, rem = c - pl * CPP, col = rem >> 3, m4 = (rem & 7) * 4;
      *reinterpret_cast<uint4*>(&Cs[pl][col][m4]) = rc[i];
    }
    __syncthreads();
    if (mb + BK < M) fetch(mb + BK);
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      const int k0 = ks * 16 + 4 * kq;
      bf8 ah[2], al[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ah[t] = ld8(&As[0][wg * 32 + t * 16 + r16][k0]);
        al[t] = ld8(&As[1][wg * 32 + t * 16 + r16][k0]);
      }
#pragma unroll
      for (int y = 0; y < YT; ++y) {
        const bf8 ch = ld8(&Cs[0][wn * 16 * YT + y * 16 + r16][k0]);
        const bf8 cl = ld8(&Cs[1][wn * 16 * YT + y * 16 + r16][k0]);
        const bf8 chn = neg_odd(ch), cln = neg_odd(cl), chs = swap(ch), cls = swap(cl);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          // Re = sum W.x C.x - W.y C.y;  Im = sum W.x C.y + W.y C.x
          accr[x][y] = acc3(ah[x], al[x], chn, cln, accr[x][y]);
          acci[x][y] = acc3(ah[x], al[x], chs, cls, acci[x][y]);
        }
      }
    }
    __syncthreads();
  }
  double dsum[YT];
#pragma unroll
  for (int y = 0; y < YT; ++y) dsum[y] = 0.0;
#pragma unroll
  for (int y = 0; y < YT; ++y) {
    const int n = n0 + wn * 16 * YT + y * 16 + r16;
    if (n >= ncols) continue;
    z64* yrow = Y.base + (long long)slots[n] * Y.stride;
    const z64* drow = dots ? dot_in.base + (long long)slots[n] * dot_in.stride : nullptr;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gg = g0 + wg * 32 + x * 16 + 4 * kq + v;
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
  for (int y = 0; y < YT; ++y) {
    dsum[y] += __shfl_xor(dsum[y], 16);
    dsum[y] += __shfl_xor(dsum[y], 32);
  }
  if (wg == 1 && kq == 0) {
#pragma unroll
    for (int y = 0; y < YT; ++y) red[y][wn * 16 + r16] = dsum[y];
  }
  __syncthreads();
  if (wg == 0 && kq == 0) {
#pragma unroll
    for (int y = 0; y < YT; ++y) {
      const int n = n0 + wn * 16 * YT + y * 16 + r16;
      if (n < ncols) dots[(long long)n * gridDim.x + tx] = dsum[y] + red[y][wn * 16 + r16];
    }
  }
}

// both bf16 planes of W (FP32 source, rows of K complex) with rows padded to ldw
__global__ void k_split_w(const z32* __restrict__ W, int M, int K, int ldw, bz* Wb,
                          long long wplane) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)M * ldw) return;
  const int m = int(i / ldw), g = int(i - (long long)m * ldw);
  const z32 v = g < K ? W[(long long)m * K + g] : z32{0.f, 0.f};
  split(v.x, v.y, Wb[i], Wb[wplane + i]);
}

// hi / lo planes of the listed FP64 vectors, Pb[plane][c][ldw] for list entry
// c (rows zero-padded past K)
__global__ void k_split_cols(VecSet<const z64> B, const int* slots, int K, int ldw, bz* Pb,
                             long long pplane) {
  const int c = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ldw) return;
  const z64 v = g < K ? B.base[(long long)slots[c] * B.stride + g] : z64{0.0, 0.0};
  const long long i = (long long)c * ldw + g;
  split(float(v.x), float(v.y), Pb[i], Pb[pplane + i]);
}

// hi / lo planes of C[c][m] (FP32), Cb[plane][c][Mp] with rows zero-padded past M
__global__ void k_split_c(const z32* __restrict__ C, int M, int Mp, bz* Cb, long long cplane) {
  const int c = blockIdx.y;
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= Mp) return;
  const z32 v = m < M ? C[(long long)c * M + m] : z32{0.f, 0.f};
  const long long i = (long long)c * Mp + m;
  split(v.x, v.y, Cb[i], Cb[cplane + i]);
}

}  // namespace

void launch_split_w(const z32* W, int M, int K, int ldw, bz* Wb, hipStream_t st) {
  const long long n = (long long)M * ldw;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_split_w, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, M, K,
                     ldw, Wb, n);
  STH_HIP_CHECK(hipGetLastError());
}

// Tile choice (environment STH_BF16_TILE): 0 = 64 x 64 tiles for both
// products; 1 (default) = 64 x 128 for Y += W C once 256 columns fill it; 2 =
// also 128 x 128 for C = W^H B.  On the 144^3 system (2048 columns, M = 2048)
// the wide Y += W C tile took 2.4% off that phase, while the 128 x 128
// C = W^H B tile, held to one wave per SIMD by its 450 registers, ran no
// faster than 64 x 64 at three.
int bf16_tile() {
  static const int t = [] {
    const char* e = std::getenv("STH_BF16_TILE");
    return e ? std::atoi(e) : 1;
  }();
  return t;
}

// the rows of W hold the columns [koff, koff + K) and every column the last
// tiles read past them (whole 64-column tiles of Y += W C, whole 32-column
// stages of C = W^H B)
static bool bf16_cols_fit(int ldw, int koff, int K) {
  return ldw % 64 == 0 && koff >= 0 && koff % 4 == 0 &&
         koff + std::max(((K + 63) / 64) * 64, K + 31) <= ldw;
}

void launch_gemm_ah_b_bf16(const bz* Wb, long long wplane, int ldw, int koff, int M,
                           VecSet<const z64> B, const int* slots, int ncols, int K, int kchunk,
                           z32* part, bz* scratch, size_t scratch_bytes, hipStream_t st) {
  if (ncols <= 0 || M <= 0) return;
  const long long pplane = (long long)ncols * ldw;
  if (!bf16_cols_fit(ldw, koff, K) || kchunk % 4 != 0 ||
      size_t(2 * pplane) * sizeof(bz) > scratch_bytes) {
    set_error("bf16 GEMM: row pitch %d, columns [%d, %d + %d), K chunk %d (multiple of 4), "
              "scratch %zu B", ldw, koff, koff, K, kchunk, scratch_bytes);
    throw Error(STH_E_INTERNAL);
  }
  Wb += koff;
  hipLaunchKernelGGL(k_split_cols, dim3((unsigned)((ldw + 255) / 256), (unsigned)ncols),
                     dim3(256), 0, st, B, slots, K, ldw, scratch, pplane);
  const int nsplit = (K + kchunk - 1) / kchunk;
  if (bf16_tile() >= 2 && ncols >= 256 && M >= 256) {
    dim3 grid((M + 127) / 128, (ncols + 127) / 128, nsplit);
    hipLaunchKernelGGL((k_gemm_ah_b_bf16<4, 4>), grid, dim3(BTHR), 0, st, Wb, wplane, ldw, M,
                       scratch, pplane, ncols, K, kchunk, part);
  } else {
    dim3 grid((M + BT - 1) / BT, (ncols + BT - 1) / BT, nsplit);
    hipLaunchKernelGGL((k_gemm_ah_b_bf16<2, 2>), grid, dim3(BTHR), 0, st, Wb, wplane, ldw, M,
                       scratch, pplane, ncols, K, kchunk, part);
  }
  STH_HIP_CHECK(hipGetLastError());
}

void launch_gemm_a_c_bf16(const bz* Wb, long long wplane, int ldw, int koff, int M, const z32* C,
                          VecSet<z64> Y, const int* slots, int ncols, int K, double s0,
                          VecSet<const z64> dot_in, double* dots, bz* scratch,
                          size_t scratch_bytes, hipStream_t st) {
  if (ncols <= 0) return;
  const int Mp = ((M + BK - 1) / BK) * BK;
  const long long cplane = (long long)ncols * Mp;
  if (!bf16_cols_fit(ldw, koff, K) || size_t(2 * cplane) * sizeof(bz) > scratch_bytes) {
    set_error("bf16 GEMM: row pitch %d, columns [%d, %d + %d), scratch %zu B", ldw, koff, koff,
              K, scratch_bytes);
    throw Error(STH_E_INTERNAL);
  }
  Wb += koff;
  if (Mp > 0)
    hipLaunchKernelGGL(k_split_c, dim3((unsigned)((Mp + 255) / 256), (unsigned)ncols),
                       dim3(256), 0, st, C, M, Mp, scratch, cplane);
  if (bf16_tile() >= 1 && ncols >= 256) {
    dim3 grid(gemm_a_c_tiles(K), (ncols + 127) / 128);
    hipLaunchKernelGGL((k_gemm_a_c_bf16<4>), grid, dim3(BTHR), 0, st, Wb, wplane, ldw, M,
                       scratch, Mp, Y, slots, ncols, K, s0, dot_in, dots);
  } else {
    dim3 grid(gemm_a_c_tiles(K), (ncols + BT - 1) / BT);
    hipLaunchKernelGGL((k_gemm_a_c_bf16<2>), grid, dim3(BTHR), 0, st, Wb, wplane, ldw, M,
                       scratch, Mp, Y, slots, ncols, K, s0, dot_in, dots);
  }
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
