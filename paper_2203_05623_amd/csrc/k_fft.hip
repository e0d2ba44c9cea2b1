// Sphere-pruned 3D FFT stages of the dual-space Hamiltonian (paper, Section 4.1:
// kinetic term in reciprocal space, local potential in real space, only the
// Fourier components inside the cutoff sphere are kept).
//
// A wave function on the sphere is carried through three kernels:
//   zfft_inv   sphere -> z-sticks: each stick (fixed m1, m2) is a line along
//              grid axis 0; its run of coefficients is placed at i0 = m0 mod N
//              and inverse-transformed.  Output layout [i0][stick] so that a
//              plane (fixed i0) of all sticks is one contiguous row.
//   plane_*    one workgroup per (vector, i0): the stick values of the plane
//              go into an N x (N + 1) LDS tile, are inverse-transformed along
//              i2 (only rows that hold sticks) and i1, multiplied by the real
//              potential, transformed forward and written back to the sticks.
//              k_plane_local does this with the forward transforms taken as
//              the adjoints of the inverse pass sequence (see there).
//   zfft_fwd   z-sticks -> sphere: forward transform along axis 0, 1/N^3, the
//              sphere components extracted, kinetic and shift terms fused.
// Every kernel is instantiated for each radix plan of its length; the plan used
// is chosen per system and precision (GridDev::plan, set by the autotuner).
// Workgroups have as many threads as the widest pass has butterflies, so each
// pass is one round of work between two barriers.
#include <algorithm>

#include <map>
#include <mutex>

#include "errors.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace sth {

namespace {

constexpr size_t kLdsBytes = 160 * 1024;   // LDS per CU on gfx950

// sticks per workgroup in the z-stick kernels: 64, halved while the LDS tile
// would exceed 40 KB
template <int N, typename T>
constexpr int zsticks() {
  int z = 64;
  while (z > 8 && z * (N + 1) * int(sizeof(cpx<T>)) > 40960) z /= 2;
  return z;
}
template <int N, int P, typename T>
constexpr int zthreads() {
  const int t = RadixPlan<N, P>::threads(zsticks<N, T>());
  return t < 256 ? 256 : t;
}
template <int N, int P>
constexpr int pthreads() {
  const int t = RadixPlan<N, P>::threads(N);
  return t < 256 ? 256 : t;
}
template <typename T>
__device__ inline const cpx<T>* twiddles(const GridDev& g);
template <>
__device__ inline const cpx<double>* twiddles<double>(const GridDev& g) { return g.tw64; }
template <>
__device__ inline const cpx<float>* twiddles<float>(const GridDev& g) { return g.tw32; }

template <typename T, typename S>
__device__ inline cpx<T> cvt(const S& v) { return cpx<T>{T(v.x), T(v.y)}; }

template <typename Z>
struct real_of;
template <typename T>
struct real_of<cpx<T>> {
  using type = T;
};

// Twiddles (and, for planes, the active-row list) are staged in LDS once per
// workgroup: the butterflies read them there instead of from global memory.
template <typename T, int NTHR>
__device__ inline void stage_twiddles(cpx<T>* dst, const cpx<T>* src, int n) {
  for (int i = threadIdx.x; i < n; i += NTHR) dst[i] = src[i];
}

// ------------------------------------------------------------------ z sticks
template <int N, int P, typename T, typename Tin>
__global__ __launch_bounds__((zthreads<N, P, T>())) void k_zfft_inv(GridDev g,
                                                                   VecSet<const Tin> in,
                                                                   VecSet<cpx<T>> sticks,
                                                                   const int* slots) {
  constexpr int NT = zthreads<N, P, T>();
  constexpr int NPAD = N + 1;
  constexpr int ZS = zsticks<N, T>();
  __shared__ cpx<T> buf[ZS * NPAD];
  __shared__ cpx<T> tw[N];
  const int slot = slots[blockIdx.y];
  const int s0 = blockIdx.x * ZS;
  const int ns = min(ZS, g.nst - s0);
  stage_twiddles<T, NT>(tw, twiddles<T>(g), N);
  for (int i = threadIdx.x; i < ZS * NPAD; i += NT) buf[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  const Tin* src = in.base + slot * in.stride;
  const int e0 = g.stick_off[s0], e1 = g.stick_off[s0 + ns];
  for (int e = e0 + threadIdx.x; e < e1; e += NT) {
    const int pos = g.elem_pos[e];
    const int st = pos / N - s0, i0 = pos - (pos / N) * N;
    buf[st * NPAD + i0] = cvt<T>(src[e]);
  }
  __syncthreads();
  RadixPlan<N, P>::template fft<T, +1, NT, ZS>::run(
      buf, ns, 1, [](int f) { return f * NPAD; }, tw);
  cpx<T>* dst = sticks.base + slot * sticks.stride;
  for (int t = threadIdx.x; t < N * ns; t += NT) {
    const int i0 = t / ns, st = t - i0 * ns;
    dst[(long long)i0 * g.nst + s0 + st] = buf[st * NPAD + i0];
  }
}

template <int N, int P, typename T, typename Tout>
__global__ __launch_bounds__((zthreads<N, P, T>())) void k_zfft_fwd(
    GridDev g, VecSet<const cpx<T>> sticks, VecSet<Tout> out, const int* slots, int mode,
    VecSet<const Tout> pin, const double* eps_slot) {
  constexpr int NT = zthreads<N, P, T>();
  constexpr int NPAD = N + 1;
  constexpr int ZS = zsticks<N, T>();
  __shared__ cpx<T> buf[ZS * NPAD];
  __shared__ cpx<T> tw[N];
  const int slot = slots[blockIdx.y];
  const int s0 = blockIdx.x * ZS;
  const int ns = min(ZS, g.nst - s0);
  stage_twiddles<T, NT>(tw, twiddles<T>(g), N);
  const cpx<T>* src = sticks.base + slot * sticks.stride;
  for (int t = threadIdx.x; t < N * ns; t += NT) {
    const int i0 = t / ns, st = t - i0 * ns;
    buf[st * NPAD + i0] = src[(long long)i0 * g.nst + s0 + st];
  }
  __syncthreads();
  RadixPlan<N, P>::template fft<T, -1, NT, ZS>::run(
      buf, ns, 1, [](int f) { return f * NPAD; }, tw);
  const double inv_n3 = 1.0 / (double(N) * N * N);
  Tout* dst = out.base + slot * out.stride;
  const int e0 = g.stick_off[s0], e1 = g.stick_off[s0 + ns];
  const double eps = (mode == ZF_SHIFT) ? eps_slot[slot] : 0.0;
  const Tout* p = (mode == ZF_SHIFT) ? pin.base + slot * pin.stride : nullptr;
  for (int e = e0 + threadIdx.x; e < e1; e += NT) {
    const int pos = g.elem_pos[e];
    const int st = pos / N - s0, i0 = pos - (pos / N) * N;
    const cpx<T> v = buf[st * NPAD + i0];
    double re = double(v.x) * inv_n3, im = double(v.y) * inv_n3;
    if (mode == ZF_SHIFT) {
      const double k = g.kin[e] - eps;
      re += k * double(p[e].x);
      im += k * double(p[e].y);
    }
    using TO = typename real_of<Tout>::type;
    dst[e].x = TO(re);
    dst[e].y = TO(im);
  }
}

// ------------------------------------------------------------------ planes
// Dynamic LDS of a plane workgroup: the N x (N + 1) tile [i1][i2], the N
// twiddles, the active-row list and, when it fits in the CU's LDS, the
// potential plane V[i1][i2].  Rows transformed along i2 are the active rows
// only (the others are zero before the i1 transform).
template <int N, typename T>
struct PlaneLds {
  static constexpr int NP = N + 1;
  static constexpr size_t base_bytes =
      size_t(N) * NP * sizeof(cpx<T>) + N * sizeof(cpx<T>) + N * sizeof(int);
  static constexpr bool kStageV = base_bytes + size_t(N) * N * sizeof(T) <= kLdsBytes;
  cpx<T>* pl;
  cpx<T>* tw;
  int* rows;
  T* v;
  __device__ explicit PlaneLds(unsigned char* raw)
      : pl(reinterpret_cast<cpx<T>*>(raw)),
        tw(reinterpret_cast<cpx<T>*>(raw) + N * NP),
        rows(reinterpret_cast<int*>(reinterpret_cast<cpx<T>*>(raw) + N * NP + N)),
        v(reinterpret_cast<T*>(raw + base_bytes)) {}
  static constexpr size_t bytes(bool with_v) {
    return base_bytes + ((with_v && kStageV) ? size_t(N) * N * sizeof(T) : 0);
  }
};

template <int N, int NT, typename T>
__device__ inline void plane_stage(PlaneLds<N, T>& L, const GridDev& g) {
  stage_twiddles<T, NT>(L.tw, twiddles<T>(g), N);
  for (int i = threadIdx.x; i < g.nrow; i += NT) L.rows[i] = g.row_list[i];
}

// inverse transform along i2 (active rows) then i1; `post` maps the outputs of
// the last pass (LDS index i1 * NP + i2)
template <int N, int P, int NT, typename T, typename Post = NoPost>
__device__ inline void plane_inverse(PlaneLds<N, T>& L, const GridDev& g, Post post = Post()) {
  constexpr int NP = N + 1;
  const int* rows = L.rows;
  RadixPlan<N, P>::template fft<T, +1, NT, N>::run(
      L.pl, g.nrow, 1, [rows](int f) { return rows[f] * NP; }, L.tw);
  RadixPlan<N, P>::template fft<T, +1, NT, N>::run(L.pl, N, NP, [](int f) { return f; }, L.tw,
                                                   post);
}

template <int N, int P, int NT, typename T>
__device__ inline void plane_forward(PlaneLds<N, T>& L, const GridDev& g) {
  constexpr int NP = N + 1;
  const int* rows = L.rows;
  RadixPlan<N, P>::template fft<T, -1, NT, N>::run(L.pl, N, NP, [](int f) { return f; }, L.tw);
  RadixPlan<N, P>::template fft<T, -1, NT, N>::run(
      L.pl, g.nrow, 1, [rows](int f) { return rows[f] * NP; }, L.tw);
}

// zero the tile, scatter the stick values of one plane (row of the stick array)
template <int N, int NT, typename T>
__device__ inline void plane_scatter(PlaneLds<N, T>& L, const GridDev& g, const cpx<T>* row) {
  constexpr int NP = N + 1;
  for (int i = threadIdx.x; i < N * NP; i += NT) L.pl[i] = cpx<T>{T(0), T(0)};
  __syncthreads();
  for (int s = threadIdx.x; s < g.nst; s += NT) {
    const int p = g.stick_i12[s];
    const int i1 = p / N, i2 = p - (p / N) * N;
    L.pl[i1 * NP + i2] = row[s];
  }
  __syncthreads();
}

// w[r] = tw[r j] = exp(-2 pi i r j / N) for r < R: w^1 read from the table, the
// other powers formed by a balanced product tree (one memory load instead of
// R - 1; each power is at most ceil(log2 R) products deep, a few ulp).
template <int R, typename T>
__device__ inline void pass_twiddles(const cpx<T>* tw, int j, cpx<T>* w) {
  w[0] = cpx<T>{T(1), T(0)};
  if constexpr (R > 1) w[1] = tw[j];
#pragma unroll
  for (int r = 2; r < R; ++r) w[r] = w[r / 2] * w[r - r / 2];
}

// Whether cell i2 of row i1 holds a stick (bit masks of the rows, N <= 128).
struct RowBits {
  unsigned long long lo, hi;
  __device__ RowBits(const GridDev& g, int i1) : lo(g.rowbits[2 * i1]), hi(g.rowbits[2 * i1 + 1]) {}
  __device__ RowBits(const unsigned long long* bits, int i1)
      : lo(bits[2 * i1]), hi(bits[2 * i1 + 1]) {}
  __device__ bool operator()(int i2) const {
    return ((i2 < 64 ? lo >> i2 : hi >> (i2 - 64)) & 1ull) != 0;
  }
};

// The stick row of plane i0 into the tile (coalesced reads; cells without a
// stick keep stale values, the first pass reads them as zero), and back.
template <int N, int NT, typename T, int NP = N + 1>
__device__ inline void sticks_to_tile(cpx<T>* tile, const GridDev& g, const cpx<T>* row) {
  for (int s = threadIdx.x; s < g.nst; s += NT) {
    const int p = g.stick_i12[s];
    const int i1 = p / N;
    tile[i1 * NP + (p - i1 * N)] = row[s];
  }
}
template <int N, int NT, typename T, int NP = N + 1>
__device__ inline void tile_to_sticks(const cpx<T>* tile, const GridDev& g, cpx<T>* row) {
  for (int s = threadIdx.x; s < g.nst; s += NT) {
    const int p = g.stick_i12[s];
    const int i1 = p / N;
    row[s] = tile[i1 * NP + (p - i1 * N)];
  }
}

// Bit i1 of the active-row mask (rows holding at least one stick).
__device__ inline bool row_active(const GridDev& g, int i1) {
  const unsigned long long m =
      i1 < 64 ? g.rowmask[0] : (i1 < 128 ? g.rowmask[1] : g.rowmask[2]);
  return (m >> (i1 & 63)) & 1ull;
}

// H_loc on one plane, single-pass form: one workgroup per (vector, i0) holding
// the whole N x (N + 1) tile.  The forward transforms are the adjoints of the
// inverse pass sequence (N = R1 R2), so the inverse pass 2 along i1, the
// potential multiply and the forward pass 2^H along i1 share one butterfly's
// registers, and every pass 2 / 2^H works in place (no barrier between its
// loads and stores):
//   A1   along i2, pass 1 on the active rows; inputs gathered from the stick row
//   A2   along i2, pass 2 on the active rows
//   B1   along i1, pass 1 on all columns; inputs from the active rows only
//   B2   along i1, pass 2, * V, pass 2^H
//   B1h  along i1, pass 1^H; outputs kept for the active rows only
//   A2h  along i2, pass 2^H on the active rows
//   A1h  along i2, pass 1^H; outputs scattered straight to the stick row
// Passes along i2 give consecutive lanes consecutive butterflies of one row,
// passes along i1 consecutive columns.
template <int N, int P>
constexpr int fused_threads() {
  return pthreads<N, P>();
}
// LDS row pitch of the single-pass tile (elements)
template <int N, typename T>
constexpr int fused_pitch() {
  return N + 1;
}
template <int N, typename T>
constexpr size_t fused_lds_bytes() {
  return size_t(N) * fused_pitch<N, T>() * sizeof(cpx<T>);
}

// The passes A1 .. A1h on the tile (stick cells already in place).  The
// plane-independent tables come in as pointers (global memory, or an LDS copy):
// rows = the active rows (row_list), bits = their stick bit masks (rowbits),
// tw = the twiddles.  vget(q, r) gives the potential at the r-th point of this
// thread's q-th B2 butterfly; after_b2() runs once the last of those values
// has been read.
template <int N, int P, typename T, typename VGet, typename AfterB2>
__device__ inline void fused_passes(cpx<T>* tile, const GridDev& g, const int* rows,
                                    const unsigned long long* bits, const cpx<T>* tw,
                                    VGet vget, AfterB2 after_b2) {
  constexpr int NT = fused_threads<N, P>();
  constexpr int NP = fused_pitch<N, T>();
  constexpr int R1 = RadixPlan<N, P>::radix(0), R2 = RadixPlan<N, P>::radix(1);
  static_assert(R1 * R2 == N, "two-pass plan");
  constexpr int M1 = N / R1, M2 = N / R2;
  constexpr int TB1 = (N * M1 + NT - 1) / NT;
  constexpr int TB2 = (N * M2 + NT - 1) / NT;
  const int nrow = g.nrow;
  {   // A1: loads, barrier, stores (in place along the row)
    constexpr int TA = (N / 2 * M1 + NT - 1) / NT;   // at most N/2 active rows
    cpx<T> v[TA][R1];
#pragma unroll
    for (int q = 0; q < TA; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < nrow * M1) {
        const int f = t / M1, j = t - f * M1;
        const int i1 = rows[f];
        const RowBits has(bits, i1);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          v[q][r] = cpx<T>{T(0), T(0)};
          if (has(j + r * M1)) v[q][r] = tile[i1 * NP + j + r * M1];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TA; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < nrow * M1) {
        const int f = t / M1, j = t - f * M1;
        const int i1 = rows[f];
        Dft<R1, +1, T>::run(v[q]);
#pragma unroll
        for (int p = 0; p < R1; ++p) tile[i1 * NP + j * R1 + p] = v[q][p];
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nrow * M2; t += NT) {   // A2
    const int j = t / nrow, f = t - j * nrow;
    const int i1 = rows[f];
    cpx<T> v[R2], w[R2];
    pass_twiddles<R2>(tw, j, w);
#pragma unroll
    for (int r = 0; r < R2; ++r) v[r] = tile[i1 * NP + j + r * M2];
#pragma unroll
    for (int r = 1; r < R2; ++r) v[r] = v[r] * conj(w[r]);
    Dft<R2, +1, T>::run(v);
#pragma unroll
    for (int q = 0; q < R2; ++q) tile[i1 * NP + j + q * M2] = v[q];
  }
  __syncthreads();
  {   // B1
    cpx<T> v[TB1][R1];
#pragma unroll
    for (int q = 0; q < TB1; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < N * M1) {
        const int j = t / N, c = t - j * N;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          const int i1 = j + r * M1;
          v[q][r] = cpx<T>{T(0), T(0)};
          if (row_active(g, i1)) v[q][r] = tile[i1 * NP + c];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TB1; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < N * M1) {
        const int j = t / N, c = t - j * N;
        Dft<R1, +1, T>::run(v[q]);
#pragma unroll
        for (int p = 0; p < R1; ++p) tile[(j * R1 + p) * NP + c] = v[q][p];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TB2; ++q) {   // B2
    const int t = threadIdx.x + q * NT;
    if (t < N * M2) {
      const int j = t / N, c = t - j * N;
      cpx<T> v[R2], w[R2];
      pass_twiddles<R2>(tw, j, w);
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = tile[(j + r * M2) * NP + c];
#pragma unroll
      for (int r = 1; r < R2; ++r) v[r] = v[r] * conj(w[r]);
      Dft<R2, +1, T>::run(v);
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = scale(v[r], vget(q, r));
      Dft<R2, -1, T>::run(v);
      tile[j * NP + c] = v[0];
#pragma unroll
      for (int r = 1; r < R2; ++r) tile[(j + r * M2) * NP + c] = v[r] * w[r];
    }
  }
  after_b2();
  __syncthreads();
  {   // B1h
    cpx<T> v[TB1][R1];
#pragma unroll
    for (int q = 0; q < TB1; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < N * M1) {
        const int j = t / N, c = t - j * N;
#pragma unroll
        for (int p = 0; p < R1; ++p) v[q][p] = tile[(j * R1 + p) * NP + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TB1; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < N * M1) {
        const int j = t / N, c = t - j * N;
        Dft<R1, -1, T>::run(v[q]);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          const int i1 = j + r * M1;
          if (row_active(g, i1)) tile[i1 * NP + c] = v[q][r];
        }
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nrow * M2; t += NT) {   // A2h
    const int j = t / nrow, f = t - j * nrow;
    const int i1 = rows[f];
    cpx<T> v[R2], w[R2];
    pass_twiddles<R2>(tw, j, w);
#pragma unroll
    for (int r = 0; r < R2; ++r) v[r] = tile[i1 * NP + j + r * M2];
    Dft<R2, -1, T>::run(v);
#pragma unroll
    for (int r = 1; r < R2; ++r) v[r] = v[r] * w[r];
#pragma unroll
    for (int r = 0; r < R2; ++r) tile[i1 * NP + j + r * M2] = v[r];
  }
  __syncthreads();
  {   // A1h: loads, barrier, stores; then the stick cells go back to the row
    constexpr int TA = (N / 2 * M1 + NT - 1) / NT;
    cpx<T> v[TA][R1];
#pragma unroll
    for (int q = 0; q < TA; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < nrow * M1) {
        const int f = t / M1, j = t - f * M1;
        const int i1 = rows[f];
#pragma unroll
        for (int p = 0; p < R1; ++p) v[q][p] = tile[i1 * NP + j * R1 + p];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TA; ++q) {
      const int t = threadIdx.x + q * NT;
      if (t < nrow * M1) {
        const int f = t / M1, j = t - f * M1;
        const int i1 = rows[f];
        Dft<R1, -1, T>::run(v[q]);
#pragma unroll
        for (int r = 0; r < R1; ++r) tile[i1 * NP + j + r * M1] = v[q][r];
      }
    }
  }
}

// Position in the B2 butterfly layout of this thread's q-th butterfly, point r:
// index of V[i1][i2] in the plane, or -1 past the end.
template <int N, int P>
__device__ inline int b2_index(int q, int r) {
  constexpr int NT = fused_threads<N, P>();
  constexpr int R2 = RadixPlan<N, P>::radix(1), M2 = N / R2;
  const int t = threadIdx.x + q * NT;
  if (t >= N * M2) return -1;
  const int j = t / N, c = t - j * N;
  return (j + r * M2) * N + c;
}

template <int N, int P, typename T>
__global__ __launch_bounds__((fused_threads<N, P>())) void k_plane_fused(
    GridDev g, VecSet<cpx<T>> sticks, const int* slots, const T* pot, const T* const* pot_ptr) {
  constexpr int NT = fused_threads<N, P>();
  constexpr int NP = fused_pitch<N, T>();
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int slot = slots[blockIdx.y];
  const int i0 = blockIdx.x;
  cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
  const T* V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
  sticks_to_tile<N, NT, T, NP>(tile, g, row);
  __syncthreads();
  fused_passes<N, P, T>(tile, g, g.row_list, g.rowbits, twiddles<T>(g),
                        [V](int q, int r) { return V[b2_index<N, P>(q, r)]; }, [] {});
  __syncthreads();
  tile_to_sticks<N, NT, T, NP>(tile, g, row);
}

// Global-address-space view of a pointer that came out of memory (a load
// through a generic pointer would be a flat load, which the barrier's LDS wait
// also waits for).
template <typename T>
__device__ inline T ld_global(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)   // the host pass of this device function has no address spaces
  return *(const __attribute__((address_space(1))) T*)(p);
#else
  return *p;
#endif
}

// Address of plane q (column q / N, plane q % N) of k_plane_fused_pf: its
// stick row and its potential plane.
template <int N, typename T>
__device__ inline void pf_plane_ptrs(const GridDev& g, VecSet<cpx<T>> sticks, const int* slots,
                                     const T* pot, const T* const* pot_ptr, long long q,
                                     cpx<T>*& row, const T*& V) {
  const int c = int(q / N), i0 = int(q - (long long)c * N);
  const int slot = slots[c];
  row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
  V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
}

// Persistent form of k_plane_fused (plane kind 3): one workgroup per CU walks
// the planes of every column with a stride of the grid size.  The single-pass
// tile fills the LDS, so the plain form has one workgroup per CU and nothing to
// hide its load latency behind; here each plane's global loads are issued one
// plane ahead into registers: the next plane's stick values as soon as the
// current ones are in the tile, its potential values as soon as the current
// B2 pass has read its own.  The loads are unconditional (lanes without a
// stick or a butterfly read element 0), so the values stay in registers.
template <int N, int P>
constexpr int pf_sticks_per_thread() {   // an alias-free sphere has < N^2 / 4 sticks
  return (N * N / 4 + fused_threads<N, P>() - 1) / fused_threads<N, P>();
}
// LDS of k_plane_fused_pf: the tile, then copies of the twiddles (N), the
// row bit masks (2 N words) and the active-row list (N / 2 entries).
template <int N, typename T>
constexpr size_t pf_lds_bytes() {
  return fused_lds_bytes<N, T>() + size_t(N) * sizeof(cpx<T>) + size_t(2 * N) * 8 +
         size_t(N / 2) * 4;
}
template <int N, int P, typename T>
__global__ __launch_bounds__((fused_threads<N, P>())) void k_plane_fused_pf(
    GridDev g, VecSet<cpx<T>> sticks, const int* __restrict__ slots, int ncols,
    const T* pot, const T* const* __restrict__ pot_ptr) {
  constexpr int NT = fused_threads<N, P>();
  constexpr int NP = fused_pitch<N, T>();
  constexpr int R2 = RadixPlan<N, P>::radix(1), M2 = N / R2;
  constexpr int TB2 = (N * M2 + NT - 1) / NT;
  constexpr int SPT = pf_sticks_per_thread<N, P>();
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  // plane-independent tables in LDS, so that the passes issue no global load
  // (a wait for one would also wait for every prefetch issued before it)
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw + fused_lds_bytes<N, T>());
  unsigned long long* bits = reinterpret_cast<unsigned long long*>(tw + N);
  int* rows = reinterpret_cast<int*>(bits + 2 * N);
  {
    const cpx<T>* gtw = twiddles<T>(g);
    for (int i = threadIdx.x; i < N; i += NT) tw[i] = gtw[i];
    for (int i = threadIdx.x; i < 2 * N; i += NT) bits[i] = g.rowbits[i];
    for (int i = threadIdx.x; i < g.nrow; i += NT) rows[i] = g.row_list[i];
  }
  // tile cell of this thread's sticks (the same for every plane); lanes past
  // the last stick take the padding cell (0, N), which no pass reads
  int pos[SPT];
#pragma unroll
  for (int k = 0; k < SPT; ++k) {
    const int s = threadIdx.x + k * NT;
    pos[k] = N;
    if (s < g.nst) {
      const int p = g.stick_i12[s];
      const int i1 = p / N;
      pos[k] = i1 * NP + (p - i1 * N);
    }
  }
  cpx<T> sv[SPT];
  T vv[TB2][R2];
  auto load_sticks = [&](const cpx<T>* row) {
#pragma unroll
    for (int k = 0; k < SPT; ++k)
      sv[k] = ld_global(row + (pos[k] != N ? threadIdx.x + k * NT : 0));
  };
  auto load_pot = [&](const T* V) {
#pragma unroll
    for (int q2 = 0; q2 < TB2; ++q2)
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int e = b2_index<N, P>(q2, r);
        vv[q2][r] = ld_global(V + (e >= 0 ? e : 0));
      }
  };
  const long long nplanes = (long long)ncols * N, step = gridDim.x;
  long long q = blockIdx.x;
  if (q >= nplanes) return;
  cpx<T>* row;
  const T* V;
  pf_plane_ptrs<N, T>(g, sticks, slots, pot, pot_ptr, q, row, V);
  load_sticks(row);
  load_pot(V);
  // The loads are issued without branches (after the last plane they fetch
  // that plane again, and the values go unused), so that every wait for them
  // is a partial one.
  for (; q < nplanes; q += step) {
    cpx<T>* nrow = row;
    const T* nV = V;
    if (q + step < nplanes)
      pf_plane_ptrs<N, T>(g, sticks, slots, pot, pot_ptr, q + step, nrow, nV);
#pragma unroll
    for (int k = 0; k < SPT; ++k) tile[pos[k]] = sv[k];
    load_sticks(nrow);
    __syncthreads();
    fused_passes<N, P, T>(tile, g, rows, bits, tw, [&vv](int q2, int r) { return vv[q2][r]; },
                          [&] { load_pot(nV); });
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SPT; ++k)
      if (pos[k] != N) row[threadIdx.x + k * NT] = tile[pos[k]];
    __syncthreads();   // the next plane's sticks overwrite the tile
    row = nrow;
    V = nV;
  }
}

// H_loc on one plane, wave form: the passes of k_plane_fused, with every
// transform owned by one wavefront.  A wave takes PW rows (passes along i2) or
// PW columns (passes along i1) and runs all passes of that direction on them;
// the exchanges between those passes stay inside the wave, so they need only a
// wave-level ordering point, and the workgroup meets at two barriers per plane
// (after the i2 inverse passes, after the i1 passes).  Waves drift apart between
// the barriers, so one wave's LDS waits overlap another's arithmetic.
// Lane mapping: lane = j * PW + q (butterfly j, transform q of the wave's group),
// so consecutive lanes take consecutive rows (LDS stride N + 1) or consecutive
// columns (stride 1, and coalesced potential reads).  (Measured on gfx950: this
// order beats butterfly-fastest lanes, whose cells are bank-disjoint on paper.)
template <int N, int P>
struct PlaneWave {
  static constexpr int R1 = RadixPlan<N, P>::radix(0), R2 = RadixPlan<N, P>::radix(1);
  static_assert(R1 * R2 == N, "two-pass plan");
  static constexpr int M1 = N / R1;   // butterflies of pass 1 per transform (= R2)
  static constexpr int M2 = N / R2;   // butterflies of pass 2 per transform (= R1)
  static constexpr int MM = M1 > M2 ? M1 : M2;
  static constexpr int PW = 64 / MM;                // transforms per wave
  static constexpr int NG = (N + PW - 1) / PW;      // column groups of a plane
  static constexpr int NW = NG < 12 ? NG : 12;      // waves per workgroup
  static constexpr int NT = NW * 64;
  static constexpr int NP = N + 1;
  static constexpr size_t lds_bytes(size_t elem) { return size_t(N) * NP * elem; }
  // register budget: one FP64 workgroup per CU (its tile takes half the LDS or
  // more), two FP32 workgroups
  template <typename T>
  static constexpr int waves_per_eu() {
    const int w = ((sizeof(T) == 4 && 2 * NW <= 24 ? 2 : 1) * NW + 3) / 4;
    return w > 8 ? 8 : w;
  }
};

// Orders the LDS accesses of one wavefront across lanes (a wave executes in
// lockstep; this only stops the compiler from moving accesses across it).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, int P, typename T>
__global__ __launch_bounds__((PlaneWave<N, P>::NT))
__attribute__((amdgpu_waves_per_eu(PlaneWave<N, P>::template waves_per_eu<T>()))) void k_plane_wave(
    GridDev g, VecSet<cpx<T>> sticks, const int* slots, const T* pot, const T* const* pot_ptr) {
  using S = PlaneWave<N, P>;
  constexpr int R1 = S::R1, R2 = S::R2, M1 = S::M1, M2 = S::M2, PW = S::PW, NW = S::NW;
  constexpr int NP = S::NP;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int slot = slots[blockIdx.y];
  const int i0 = blockIdx.x;
  cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
  const T* V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
  const cpx<T>* tw = twiddles<T>(g);
  const int nrow = g.nrow;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // lane = j * PW + q: butterfly j of transform q of the wave's group
  const int j1 = lane / PW, q1 = lane - j1 * PW;
  const int j2 = j1, q2 = q1;
  // the passes that touch the stick row take lane = q * M1 + j instead, so that
  // consecutive lanes read and write consecutive sticks of one row
  const int qg = lane / M1, jg = lane - qg * M1;
  const int nga = (nrow + PW - 1) / PW;

  sticks_to_tile<N, S::NT, T>(tile, g, row);
  __syncthreads();
  // along i2, inverse: A1 then A2 on the wave's rows
  for (int grp = wave; grp < nga; grp += NW) {
    const int fg = grp * PW + qg, f2 = grp * PW + q2;
    const bool a1 = qg < PW && fg < nrow;
    const int ig = a1 ? g.row_list[fg] : 0;
    cpx<T> v[R1];
    if (a1) {
      const RowBits has(g, ig);
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        v[r] = cpx<T>{T(0), T(0)};
        if (has(jg + r * M1)) v[r] = tile[ig * NP + jg + r * M1];
      }
    }
    wave_sync();
    if (a1) {
      Dft<R1, +1, T>::run(v);
#pragma unroll
      for (int q = 0; q < R1; ++q) tile[ig * NP + jg * R1 + q] = v[q];
    }
    wave_sync();
    if (j2 < M2 && f2 < nrow) {
      const int i1 = g.row_list[f2];
      cpx<T> v[R2], w[R2];
      pass_twiddles<R2>(tw, j2, w);
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = tile[i1 * NP + j2 + r * M2];
#pragma unroll
      for (int r = 1; r < R2; ++r) v[r] = v[r] * conj(w[r]);
      Dft<R2, +1, T>::run(v);
#pragma unroll
      for (int q = 0; q < R2; ++q) tile[i1 * NP + j2 + q * M2] = v[q];
    }
    wave_sync();
  }
  __syncthreads();

  // along i1: pass 1, pass 2 * V * pass 2^H, pass 1^H on the wave's columns
  for (int grp = wave; grp < S::NG; grp += NW) {
    const int c1 = grp * PW + q1, c2 = grp * PW + q2;
    const bool b1 = j1 < M1 && c1 < N;
    const bool b2 = j2 < M2 && c2 < N;
    cpx<T> v[R1];
    if (b1) {
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int i1 = j1 + r * M1;
        v[r] = cpx<T>{T(0), T(0)};
        if (row_active(g, i1)) v[r] = tile[i1 * NP + c1];
      }
    }
    wave_sync();
    if (b1) {
      Dft<R1, +1, T>::run(v);
#pragma unroll
      for (int p = 0; p < R1; ++p) tile[(j1 * R1 + p) * NP + c1] = v[p];
    }
    wave_sync();
    if (b2) {
      cpx<T> u[R2], w[R2];
      pass_twiddles<R2>(tw, j2, w);
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = tile[(j2 + r * M2) * NP + c2];
#pragma unroll
      for (int r = 1; r < R2; ++r) u[r] = u[r] * conj(w[r]);
      Dft<R2, +1, T>::run(u);
#pragma unroll
      for (int r = 0; r < R2; ++r) u[r] = scale(u[r], V[(j2 + r * M2) * N + c2]);
      Dft<R2, -1, T>::run(u);
      tile[j2 * NP + c2] = u[0];
#pragma unroll
      for (int r = 1; r < R2; ++r) tile[(j2 + r * M2) * NP + c2] = u[r] * w[r];
    }
    wave_sync();
    if (b1) {
#pragma unroll
      for (int p = 0; p < R1; ++p) v[p] = tile[(j1 * R1 + p) * NP + c1];
    }
    wave_sync();
    if (b1) {
      Dft<R1, -1, T>::run(v);
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        const int i1 = j1 + r * M1;
        if (row_active(g, i1)) tile[i1 * NP + c1] = v[r];
      }
    }
    wave_sync();
  }
  __syncthreads();

  // along i2, forward: A2h then A1h on the wave's rows
  for (int grp = wave; grp < nga; grp += NW) {
    const int fg = grp * PW + qg, f2 = grp * PW + q2;
    if (j2 < M2 && f2 < nrow) {
      const int i1 = g.row_list[f2];
      cpx<T> v[R2], w[R2];
      pass_twiddles<R2>(tw, j2, w);
#pragma unroll
      for (int r = 0; r < R2; ++r) v[r] = tile[i1 * NP + j2 + r * M2];
      Dft<R2, -1, T>::run(v);
#pragma unroll
      for (int r = 1; r < R2; ++r) v[r] = v[r] * w[r];
#pragma unroll
      for (int r = 0; r < R2; ++r) tile[i1 * NP + j2 + r * M2] = v[r];
    }
    wave_sync();
    const bool a1 = qg < PW && fg < nrow;
    const int ig = a1 ? g.row_list[fg] : 0;
    cpx<T> v[R1];
    if (a1) {
#pragma unroll
      for (int p = 0; p < R1; ++p) v[p] = tile[ig * NP + jg * R1 + p];
    }
    wave_sync();
    if (a1) {
      Dft<R1, -1, T>::run(v);
#pragma unroll
      for (int r = 0; r < R1; ++r) tile[ig * NP + jg + r * M1] = v[r];
    }
    wave_sync();
  }
  __syncthreads();
  tile_to_sticks<N, S::NT, T>(tile, g, row);
}

// ------------------------------------------------------------------ z sticks, wave form
// The z-stick transforms with every stick owned by one wavefront (the lane
// mapping and the passes of k_plane_wave along i2): a wave zero-fills, fills and
// transforms its PW sticks with only wave-level ordering; the workgroup meets
// once, around the transposed exchange with the [i0][stick] array.
template <int N, int P, typename T>
struct ZWave {
  using S = PlaneWave<N, P>;
  static constexpr int NWZ = sizeof(T) == 8 ? 5 : 10;   // waves per workgroup
  static constexpr int ZS = NWZ * S::PW;                // sticks per workgroup
  static constexpr int NT = NWZ * 64;
  static constexpr int NP = N + 1;
};

template <int N, int P, typename T, typename Tin>
__global__ __launch_bounds__((ZWave<N, P, T>::NT)) void k_zfft_inv_wave(GridDev g,
                                                                       VecSet<const Tin> in,
                                                                       VecSet<cpx<T>> sticks,
                                                                       const int* slots) {
  using Z = ZWave<N, P, T>;
  using S = PlaneWave<N, P>;
  constexpr int R1 = S::R1, R2 = S::R2, M1 = S::M1, M2 = S::M2, PW = S::PW;
  constexpr int ZS = Z::ZS, NP = Z::NP, NT = Z::NT;
  __shared__ cpx<T> buf[ZS * NP];
  const int slot = slots[blockIdx.y];
  const int s0 = blockIdx.x * ZS;
  const int ns = min(ZS, g.nst - s0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane / PW, q = lane - j * PW;
  const int sw = wave * PW;                    // first stick of the wave (local)
  const int nw = max(0, min(PW, ns - sw));     // sticks of the wave
  const cpx<T>* tw = twiddles<T>(g);
  // zero-fill and fill the wave's sticks
  for (int e = lane; e < nw * N; e += 64) {
    const int st = e / N;
    buf[(sw + st) * NP + (e - st * N)] = cpx<T>{T(0), T(0)};
  }
  wave_sync();
  const Tin* src = in.base + slot * in.stride;
  if (nw > 0) {
    const int e0 = g.stick_off[s0 + sw], e1 = g.stick_off[s0 + sw + nw];
    for (int e = e0 + lane; e < e1; e += 64) {
      const int pos = g.elem_pos[e];
      const int st = pos / N - s0, i0 = pos - (pos / N) * N;
      buf[st * NP + i0] = cvt<T>(src[e]);
    }
  }
  wave_sync();
  const bool live = q < nw;
  const int st = sw + q;
  cpx<T> v[R1];
  if (live && j < M1) {
#pragma unroll
    for (int r = 0; r < R1; ++r) v[r] = buf[st * NP + j + r * M1];
  }
  wave_sync();
  if (live && j < M1) {
    Dft<R1, +1, T>::run(v);
#pragma unroll
    for (int p = 0; p < R1; ++p) buf[st * NP + j * R1 + p] = v[p];
  }
  wave_sync();
  if (live && j < M2) {
    cpx<T> u[R2], w[R2];
    pass_twiddles<R2>(tw, j, w);
#pragma unroll
    for (int r = 0; r < R2; ++r) u[r] = buf[st * NP + j + r * M2];
#pragma unroll
    for (int r = 1; r < R2; ++r) u[r] = u[r] * conj(w[r]);
    Dft<R2, +1, T>::run(u);
#pragma unroll
    for (int r = 0; r < R2; ++r) buf[st * NP + j + r * M2] = u[r];
  }
  __syncthreads();
  cpx<T>* dst = sticks.base + slot * sticks.stride;
  for (int t = threadIdx.x; t < N * ns; t += NT) {
    const int i0 = t / ns, sl = t - i0 * ns;
    dst[(long long)i0 * g.nst + s0 + sl] = buf[sl * NP + i0];
  }
}

template <int N, int P, typename T, typename Tout>
__global__ __launch_bounds__((ZWave<N, P, T>::NT)) void k_zfft_fwd_wave(
    GridDev g, VecSet<const cpx<T>> sticks, VecSet<Tout> out, const int* slots, int mode,
    VecSet<const Tout> pin, const double* eps_slot) {
  using Z = ZWave<N, P, T>;
  using S = PlaneWave<N, P>;
  constexpr int R1 = S::R1, R2 = S::R2, M1 = S::M1, M2 = S::M2, PW = S::PW;
  constexpr int ZS = Z::ZS, NP = Z::NP, NT = Z::NT;
  __shared__ cpx<T> buf[ZS * NP];
  const int slot = slots[blockIdx.y];
  const int s0 = blockIdx.x * ZS;
  const int ns = min(ZS, g.nst - s0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane / PW, q = lane - j * PW;
  const int sw = wave * PW;
  const int nw = max(0, min(PW, ns - sw));
  const cpx<T>* tw = twiddles<T>(g);
  const cpx<T>* src = sticks.base + slot * sticks.stride;
  for (int t = threadIdx.x; t < N * ns; t += NT) {
    const int i0 = t / ns, sl = t - i0 * ns;
    buf[sl * NP + i0] = src[(long long)i0 * g.nst + s0 + sl];
  }
  __syncthreads();
  // forward transform as the adjoint of the inverse passes: pass 2^H, pass 1^H
  const bool live = q < nw;
  const int st = sw + q;
  if (live && j < M2) {
    cpx<T> u[R2], w[R2];
    pass_twiddles<R2>(tw, j, w);
#pragma unroll
    for (int r = 0; r < R2; ++r) u[r] = buf[st * NP + j + r * M2];
    Dft<R2, -1, T>::run(u);
#pragma unroll
    for (int r = 1; r < R2; ++r) u[r] = u[r] * w[r];
#pragma unroll
    for (int r = 0; r < R2; ++r) buf[st * NP + j + r * M2] = u[r];
  }
  wave_sync();
  cpx<T> v[R1];
  if (live && j < M1) {
#pragma unroll
    for (int p = 0; p < R1; ++p) v[p] = buf[st * NP + j * R1 + p];
  }
  wave_sync();
  if (live && j < M1) {
    Dft<R1, -1, T>::run(v);
#pragma unroll
    for (int r = 0; r < R1; ++r) buf[st * NP + j + r * M1] = v[r];
  }
  wave_sync();
  // the wave's sticks back to the sphere, with 1/N^3 and the kinetic / shift term
  if (nw == 0) return;
  const double inv_n3 = 1.0 / (double(N) * N * N);
  Tout* dst = out.base + slot * out.stride;
  const double eps = (mode == ZF_SHIFT) ? eps_slot[slot] : 0.0;
  const Tout* p = (mode == ZF_SHIFT) ? pin.base + slot * pin.stride : nullptr;
  const int e0 = g.stick_off[s0 + sw], e1 = g.stick_off[s0 + sw + nw];
  for (int e = e0 + lane; e < e1; e += 64) {
    const int pos = g.elem_pos[e];
    const int sl = pos / N - s0, i0 = pos - (pos / N) * N;
    const cpx<T> c = buf[sl * NP + i0];
    double re = double(c.x) * inv_n3, im = double(c.y) * inv_n3;
    if (mode == ZF_SHIFT) {
      const double k = g.kin[e] - eps;
      re += k * double(p[e].x);
      im += k * double(p[e].y);
    }
    using TO = typename real_of<Tout>::type;
    dst[e].x = TO(re);
    dst[e].y = TO(im);
  }
}

template <int N, int P, typename T>
__global__ __launch_bounds__((pthreads<N, P>())) void k_plane_to_grid(
    GridDev g, VecSet<const cpx<T>> sticks, VecSet<cpx<T>> grid, const int* slots) {
  constexpr int NT = pthreads<N, P>();
  constexpr int NP = N + 1;
  extern __shared__ unsigned char smem_raw[];
  PlaneLds<N, T> L(smem_raw);
  const int slot = slots[blockIdx.y];
  const int i0 = blockIdx.x;
  const cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
  plane_stage<N, NT, T>(L, g);
  plane_scatter<N, NT, T>(L, g, row);
  plane_inverse<N, P, NT, T>(L, g);
  cpx<T>* dst = grid.base + slot * grid.stride + (long long)i0 * N * N;
  for (int e = threadIdx.x; e < N * N; e += NT) {
    const int i1 = e / N, i2 = e - (e / N) * N;
    dst[e] = L.pl[i1 * NP + i2];
  }
}

// Delta n for perturbation j = blockIdx.y on plane i0 = blockIdx.x, summed over the
// bands in a fixed order (deterministic, no atomics).
template <int N, int P>
__global__ __launch_bounds__((pthreads<N, P>())) void k_drho(GridDev g, const z64* sticks,
                                                            long long sstride, int nband,
                                                            const int* bands, const z64* psir,
                                                            double coef, double* drho) {
  constexpr int NT = pthreads<N, P>();
  constexpr int NP = N + 1;
  constexpr int PER = (N * N + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  PlaneLds<N, double> L(smem_raw);
  const int j = blockIdx.y, i0 = blockIdx.x;
  const long long n3 = (long long)N * N * N;
  plane_stage<N, NT, double>(L, g);
  double acc[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0.0;
  for (int v = 0; v < nband; ++v) {
    const z64* row = sticks + ((long long)j * nband + v) * sstride + (long long)i0 * g.nst;
    plane_scatter<N, NT, double>(L, g, row);
    plane_inverse<N, P, NT, double>(L, g);
    const z64* pr = psir + (long long)bands[v] * n3 + (long long)i0 * N * N;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < N * N) {
        const int i1 = e / N, i2 = e - (e / N) * N;
        const z64 a = pr[e], d = L.pl[i1 * NP + i2];
        acc[q] += a.x * d.x + a.y * d.y;
      }
    }
    __syncthreads();
  }
  double* out = drho + (long long)j * n3 + (long long)i0 * N * N;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NT;
    if (e < N * N) out[e] = coef * acc[q];
  }
}

// ------------------------------------------------------------------ planes in strips
// Plane form for grids whose N x (N + 1) tile exceeds the LDS (N = 144: 334 KB
// in FP64), also selectable on the smaller grids.  A plane is processed in
// strips: strips of active rows for the transforms along i2 and strips of CC
// columns for the transforms along i1, passed through a scratch plane
// Y[nrow][N] (active rows only) in global memory.  The grid is persistent: at
// most g.stage_slots workgroups, each looping over planes with its own scratch
// plane, so the scratch of the whole grid (stage_slots x nrow x N values) is
// rewritten in place and stays in the caches.  Each strip is read and written
// coalesced (rows: consecutive i2; columns: runs of CC consecutive i2).
constexpr size_t kStripTileBudget = 58 * 1024;   // LDS of a strip tile: two workgroups per CU
// rows per strip (an alias-free sphere has at most N/2 active rows)
template <int N, typename T>
constexpr int strip_rows() {
  int r = N / 2;
  while (r > 1 && size_t(r) * (N + 1) * sizeof(cpx<T>) > kStripTileBudget) --r;
  return r;
}
// columns per strip: the largest divisor of N whose strip fits
template <int N, typename T>
constexpr int strip_cols() {
  int c = N;
  while (c > 1 && (N % c != 0 || size_t(N) * (c + 1) * sizeof(cpx<T>) > kStripTileBudget)) --c;
  return c;
}
template <int N, typename T>
struct Strips {
  static constexpr int NT = 512;
  static constexpr int NP = N + 1;
  static constexpr int RC = strip_rows<N, T>();
  static constexpr int CC = strip_cols<N, T>();
  static constexpr int CP = CC + 1;               // LDS pitch of a column strip
  static constexpr int NCS = N / CC;              // column strips of a plane
  static constexpr size_t tile_elems = size_t(RC) * NP > size_t(N) * CP ? size_t(RC) * NP
                                                                         : size_t(N) * CP;
  static constexpr size_t tile_bytes = tile_elems * sizeof(cpx<T>);
  static constexpr size_t lds_bytes = tile_bytes + N * sizeof(cpx<T>) + N * sizeof(int);
};

// rows per strip when nrow rows are split into the fewest strips of <= rc rows
__device__ inline int strip_rows_balanced(int nrow, int rc) {
  const int ns = (nrow + rc - 1) / rc;
  return (nrow + ns - 1) / ns;
}

// LDS of a strip-form workgroup: strip tile, twiddles, row index (i1 -> position
// in the active-row list, -1 for an empty row).
template <int N, typename T>
struct StripLds {
  cpx<T>* tile;
  cpx<T>* tw;
  int* rowidx;
  __device__ StripLds(unsigned char* raw, const GridDev& g) {
    using S = Strips<N, T>;
    tile = reinterpret_cast<cpx<T>*>(raw);
    tw = reinterpret_cast<cpx<T>*>(raw + S::tile_bytes);
    rowidx = reinterpret_cast<int*>(raw + S::tile_bytes + N * sizeof(cpx<T>));
    stage_twiddles<T, S::NT>(tw, twiddles<T>(g), N);
    for (int i = threadIdx.x; i < N; i += S::NT) rowidx[i] = -1;
    __syncthreads();
    for (int i = threadIdx.x; i < g.nrow; i += S::NT) rowidx[g.row_list[i]] = i;
    __syncthreads();
  }
};

// stick row of a plane -> inverse along i2 on the active rows -> Y
template <int N, int P, typename T>
__device__ inline void strips_rows_inverse(const StripLds<N, T>& L, const GridDev& g,
                                           const cpx<T>* row, cpx<T>* Y) {
  using S = Strips<N, T>;
  constexpr int NT = S::NT, NP = S::NP, RC = S::RC;
  const int rs = strip_rows_balanced(g.nrow, RC);
  for (int r0 = 0; r0 < g.nrow; r0 += rs) {
    const int nr = min(rs, g.nrow - r0);
    for (int i = threadIdx.x; i < nr * NP; i += NT) L.tile[i] = cpx<T>{T(0), T(0)};
    __syncthreads();
    for (int s = threadIdx.x; s < g.nst; s += NT) {
      const int p = g.stick_i12[s];
      const int i1 = p / N;
      const int rr = L.rowidx[i1] - r0;
      if (rr >= 0 && rr < nr) L.tile[rr * NP + (p - i1 * N)] = row[s];
    }
    __syncthreads();
    RadixPlan<N, P>::template fft<T, +1, NT, RC>::run(
        L.tile, nr, 1, [](int f) { return f * NP; }, L.tw);
    for (int i = threadIdx.x; i < nr * N; i += NT) {
      const int rr = i / N, i2 = i - rr * N;
      Y[(long long)(r0 + rr) * N + i2] = L.tile[rr * NP + i2];
    }
    __syncthreads();
  }
}

// Y -> forward along i2 on the active rows -> stick row of the plane
template <int N, int P, typename T>
__device__ inline void strips_rows_forward(const StripLds<N, T>& L, const GridDev& g,
                                           const cpx<T>* Y, cpx<T>* row) {
  using S = Strips<N, T>;
  constexpr int NT = S::NT, NP = S::NP, RC = S::RC;
  const int rs = strip_rows_balanced(g.nrow, RC);
  for (int r0 = 0; r0 < g.nrow; r0 += rs) {
    const int nr = min(rs, g.nrow - r0);
    for (int i = threadIdx.x; i < nr * N; i += NT) {
      const int rr = i / N, i2 = i - rr * N;
      L.tile[rr * NP + i2] = Y[(long long)(r0 + rr) * N + i2];
    }
    __syncthreads();
    RadixPlan<N, P>::template fft<T, -1, NT, RC>::run(
        L.tile, nr, 1, [](int f) { return f * NP; }, L.tw);
    for (int s = threadIdx.x; s < g.nst; s += NT) {
      const int p = g.stick_i12[s];
      const int i1 = p / N;
      const int rr = L.rowidx[i1] - r0;
      if (rr >= 0 && rr < nr) row[s] = L.tile[rr * NP + (p - i1 * N)];
    }
    __syncthreads();
  }
}

// columns c0 .. c0 + CC of Y (active rows, zero elsewhere) -> tile [i1][cc]
// (pitch CP), inverse along i1; `post` maps the outputs of the last pass
template <int N, int P, typename T, typename Post = NoPost>
__device__ inline void strips_cols_inverse(const StripLds<N, T>& L, const cpx<T>* Y, int c0,
                                           Post post = Post()) {
  using S = Strips<N, T>;
  constexpr int NT = S::NT, CC = S::CC, CP = S::CP;
  for (int i = threadIdx.x; i < N * CC; i += NT) {
    const int i1 = i / CC, cc = i - i1 * CC;
    const int r = L.rowidx[i1];
    cpx<T> v = cpx<T>{T(0), T(0)};
    if (r >= 0) v = Y[(long long)r * N + c0 + cc];
    L.tile[i1 * CP + cc] = v;
  }
  __syncthreads();
  RadixPlan<N, P>::template fft<T, +1, NT, CC>::run(
      L.tile, CC, CP, [](int f) { return f; }, L.tw, post);
}

// multiplies the outputs of the last inverse pass along i1 by V[i1][c0 + cc]
template <int N, int CP, typename T>
struct MulPot {
  const T* V;
  int c0;
  __device__ cpx<T> operator()(int a, cpx<T> v) const {
    const int i1 = a / CP, cc = a - i1 * CP;
    const T x = V[i1 * N + c0 + cc];
    return cpx<T>{v.x * x, v.y * x};
  }
};

// H_loc (or Delta V_j) on every plane of ncols vectors
template <int N, int P, typename T>
__global__ __launch_bounds__((Strips<N, T>::NT)) void k_plane_strips(
    GridDev g, VecSet<cpx<T>> sticks, const int* slots, int ncols, const T* pot,
    const T* const* pot_ptr, cpx<T>* scratch) {
  using S = Strips<N, T>;
  constexpr int NT = S::NT, CC = S::CC, CP = S::CP;
  extern __shared__ unsigned char smem_raw[];
  const StripLds<N, T> L(smem_raw, g);
  cpx<T>* Y = scratch + (long long)blockIdx.x * g.nrow * N;
  const long long nplanes = (long long)ncols * N;
  for (long long q = blockIdx.x; q < nplanes; q += gridDim.x) {
    const int c = int(q / N), i0 = int(q - (long long)c * N);
    const int slot = slots[c];
    cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
    const T* V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
    strips_rows_inverse<N, P, T>(L, g, row, Y);
    for (int c0 = 0; c0 < N; c0 += CC) {
      strips_cols_inverse<N, P, T>(L, Y, c0, MulPot<N, CP, T>{V, c0});
      RadixPlan<N, P>::template fft<T, -1, NT, CC>::run(
          L.tile, CC, CP, [](int f) { return f; }, L.tw);
      for (int i = threadIdx.x; i < g.nrow * CC; i += NT) {
        const int r = i / CC, cc = i - r * CC;
        Y[(long long)r * N + c0 + cc] = L.tile[g.row_list[r] * CP + cc];
      }
      __syncthreads();
    }
    strips_rows_forward<N, P, T>(L, g, Y, row);
  }
}

// ------------------------------------------------------------------ compact-row planes
// Plane form that keeps only the active rows of a plane, Y[f][i2] for the nrow
// rows f of row_list, in LDS (nrow x N complex, no padding: 71 x 144 FP64 is
// 163,584 B), so that no scratch plane goes through HBM.  Every length-N
// transform runs in the registers of a group of L lanes (N = L R): lane l holds
// the elements l + L r (r < R), takes the radix-R DFT over r in its registers,
// the twiddles w_N^(l p), and a radix-2 network of log2 L stages across the
// lanes of its group (DPP lane selects, no LDS).  LDS is only the exchange between the
// row transforms (along i2) and the column transforms (along i1).
//
// Index algebra (n = l + L r, k = p + R q): X[p + R q] =
//   sum_l w_L^(l q) w_N^(l p) sum_r x[l + L r] w_R^(r p);
// the lane network is decimation in frequency (natural order in, lane
// bitrev(q) holding q out) for the inverse transform, and its adjoint,
// decimation in time (bit-reversed in, natural out), for the forward one.
//
// LDS rows are rotated by their index (element c of row f at f N + (c + f) mod N),
// so that the L lanes of a column transform, which read L consecutive rows of
// one column, hit distinct banks.
template <int N, typename T>
struct RowsForm {
  static constexpr int L = (N % 16 == 0) ? 16 : 8;   // lanes per transform
  static constexpr int R = N / L;                      // elements per lane
  static constexpr int LOG2L = L == 16 ? 4 : 3;
  // groups of L lanes per workgroup, so that the N columns split evenly; the
  // FP32 144^3 plane (81,792 B) takes 16 groups, so that two workgroups (LDS
  // and registers) share a CU
  static constexpr int G = N == 144 ? (sizeof(T) == 4 ? 16 : 36)
                                    : (N == 96 ? 48 : (N == 72 ? 72 : (N == 48 ? 48 : 24)));
  static constexpr int NT = G * L;
  static_assert(NT % 64 == 0 && NT <= 1024, "workgroup shape");
  static_assert(R == 3 || R == 6 || R == 9, "in-lane radix");
};

// LDS bytes of the compact-row form for a grid with nrow active rows
template <int N, typename T>
inline size_t rows_lds_bytes(int nrow) {
  return size_t(nrow) * N * sizeof(cpx<T>);
}

// Position of row i1 in the (ascending) active-row list, -1 for an empty row:
// a popcount of the row mask below i1 (N <= 192), so that no table takes LDS.
__device__ inline int compact_row(const GridDev& g, int i1) {
  const int w = i1 >> 6, b = i1 & 63;
  const unsigned long long mw = w == 0 ? g.rowmask[0] : (w == 1 ? g.rowmask[1] : g.rowmask[2]);
  if (((mw >> b) & 1ull) == 0) return -1;
  int f = __popcll(mw & ((1ull << b) - 1ull));
  if (w >= 1) f += __popcll(g.rowmask[0]);
  if (w >= 2) f += __popcll(g.rowmask[1]);
  return f;
}

template <int N>
__device__ inline int rows_rot(int f, int c) {
  const int x = c + f;
  return x >= N ? x - N : x;
}

// Value of lane l ^ m (m = 1, 2, 4, 8) through DPP lane selects in the vector
// ALU instead of the LDS crossbar: xor 1 and xor 2 are quad permutations, xor 8
// is a rotation by 8 of a 16-lane row, xor 4 reverses each quad and then each
// half-row (i -> i ^ 3 -> i ^ 3 ^ 7).
template <int CTRL>
__device__ inline int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dpp_sel(float v) {
  return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ inline double dpp_sel(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = unsigned(dpp32<CTRL>(int(unsigned(b))));
  const unsigned hi = unsigned(dpp32<CTRL>(int(unsigned(b >> 32))));
  return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
template <typename T>
__device__ inline T lane_xor1(T v, int m) {
  constexpr int kQuadSwap1 = 0xB1;      // quad_perm [1, 0, 3, 2]
  constexpr int kQuadSwap2 = 0x4E;      // quad_perm [2, 3, 0, 1]
  constexpr int kQuadReverse = 0x1B;    // quad_perm [3, 2, 1, 0]
  constexpr int kRowHalfMirror = 0x141;
  constexpr int kRowRor8 = 0x128;
  switch (m) {
    case 1: return dpp_sel<kQuadSwap1>(v);
    case 2: return dpp_sel<kQuadSwap2>(v);
    case 4: return dpp_sel<kRowHalfMirror>(dpp_sel<kQuadReverse>(v));
    default: return dpp_sel<kRowRor8>(v);
  }
}
template <typename T>
__device__ inline cpx<T> lane_xor(cpx<T> v, int m) {
  return cpx<T>{lane_xor1(v.x, m), lane_xor1(v.y, m)};
}

// Length-N transform held by a lane group.  inverse(): natural element order
// (lane l, register r = element l + L r) to lane l, register p = element
// p + R bitrev(l).  forward(): the adjoint, that layout back to natural order.
// tw: the table exp(-2 pi i t / N).
template <int N, typename T>
struct LaneFFT {
  using F = RowsForm<N, T>;
  static constexpr int L = F::L, R = F::R;
  __device__ static int bitrev(int l) {
    return int(__builtin_bitreverse32(unsigned(l)) >> (32 - F::LOG2L));
  }
  __device__ static void inverse(cpx<T> (&v)[R], const cpx<T>* tw, int l) {
    Dft<R, +1, T>::run(v);
    cpx<T> w[R];
    pass_twiddles<R>(tw, l, w);   // w[p] = w_N^(-l p); the inverse takes the conjugates
#pragma unroll
    for (int p = 1; p < R; ++p) v[p] = v[p] * conj(w[p]);
    // decimation in frequency, sign +: the top lane of a pair keeps a + b, the
    // bottom one (a - b) w; both as (u + s v) w_s with s = +1, w_s = 1 on top
    // and s = -1, w_s = w below (no select, one instruction stream)
#pragma unroll
    for (int h = L / 2; h >= 1; h >>= 1) {
      const bool bottom = (l & h) != 0;
      const T sg = bottom ? T(-1) : T(1);
      const cpx<T> wt = conj(tw[(l & (h - 1)) * (N / (2 * h))]);
      const cpx<T> ws = bottom ? wt : cpx<T>{T(1), T(0)};
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const cpx<T> u = lane_xor(v[p], h);
        v[p] = cpx<T>{u.x + sg * v[p].x, u.y + sg * v[p].y} * ws;
      }
    }
  }
  __device__ static void forward(cpx<T> (&v)[R], const cpx<T>* tw, int l) {
    // decimation in time, sign -: top a + b w, bottom a - b w.  Each lane
    // scales its own value first (the bottom one by w, the top one by 1) and
    // exchanges the product: z_partner + s z_self with s = +1 on top, -1 below.
#pragma unroll
    for (int h = 1; h < L; h <<= 1) {
      const bool bottom = (l & h) != 0;
      const T sg = bottom ? T(-1) : T(1);
      const cpx<T> wt = tw[(l & (h - 1)) * (N / (2 * h))];
      const cpx<T> ws = bottom ? wt : cpx<T>{T(1), T(0)};
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const cpx<T> z = v[p] * ws;
        const cpx<T> zp = lane_xor(z, h);
        v[p] = cpx<T>{zp.x + sg * z.x, zp.y + sg * z.y};
      }
    }
    cpx<T> w[R];
    pass_twiddles<R>(tw, l, w);
#pragma unroll
    for (int p = 1; p < R; ++p) v[p] = v[p] * w[p];
    Dft<R, -1, T>::run(v);
  }
};

// H_loc (or Delta V_j) on every plane of ncols vectors, compact-row form
// (plane kind 4).  Persistent grid: one workgroup per CU walks the planes.
// Per plane: (A) each lane group takes rows f (f = group, group + G, ...):
// clears its row, scatters the row's sticks into it (the sticks of one row are
// a contiguous range), inverse transform along i2, back to the row; (B) each
// group takes columns: gathers the active rows of the column, inverse along
// i1, multiplies by V, forward along i1, writes the active rows back; (C)
// the row groups again: forward along i2, stick cells back to the stick row.
// A group touches only its own rows in (A) and (C), so the LDS writes and
// reads of one row stay inside one wavefront (in order); two workgroup
// barriers per plane separate (A), (B) and (C).
template <int N, typename T>
__global__ __launch_bounds__((RowsForm<N, T>::NT)) void k_plane_rows(
    GridDev g, VecSet<cpx<T>> sticks, const int* __restrict__ slots, int ncols, const T* pot,
    const T* const* __restrict__ pot_ptr) {
  using F = RowsForm<N, T>;
  using X = LaneFFT<N, T>;
  constexpr int L = F::L, R = F::R, G = F::G;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* Y = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nrow = g.nrow;
  const int l = threadIdx.x % L, grp = threadIdx.x / L;
  const int lq = X::bitrev(l);
  // compact row (+1, 0 for an empty row) of each i1 = l + L r this lane holds in
  // a column transform, one byte each
  unsigned fpk[(R + 3) / 4];
#pragma unroll
  for (int i = 0; i < (R + 3) / 4; ++i) fpk[i] = 0u;
#pragma unroll
  for (int r = 0; r < R; ++r)
    fpk[r >> 2] |= unsigned(compact_row(g, l + L * r) + 1) << (8 * (r & 3));
  auto fof = [&](int r) { return int((fpk[r >> 2] >> (8 * (r & 3))) & 0xFFu) - 1; };
  const long long nplanes = (long long)ncols * N;
  for (long long q = blockIdx.x; q < nplanes; q += gridDim.x) {
    // the twiddle pointer is opaque to the compiler per plane (an empty asm
    // that claims to change it), so that the twiddle loads are redone per
    // plane from the cache instead of being hoisted out of the loop into
    // registers that would have to be spilled
    const cpx<T>* tw = twiddles<T>(g);
    asm volatile("" : "+s"(tw));
    const int c = int(q / N), i0 = int(q - (long long)c * N);
    const int slot = slots[c];
    cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
    const T* V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
    // (A) rows, inverse along i2
    for (int f = grp; f < nrow; f += G) {
      cpx<T>* yr = Y + f * N;
#pragma unroll
      for (int r = 0; r < R; ++r) yr[l + L * r] = cpx<T>{T(0), T(0)};
      const int s1 = g.row_srange[2 * f + 1];
      for (int s = g.row_srange[2 * f] + l; s < s1; s += L) {
        const int i2 = g.stick_i12[s] % N;
        yr[rows_rot<N>(f, i2)] = row[s];
      }
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = yr[rows_rot<N>(f, l + L * r)];
      X::inverse(v, tw, l);
#pragma unroll
      for (int p = 0; p < R; ++p) yr[rows_rot<N>(f, p + R * lq)] = v[p];
    }
    __syncthreads();
    // (B) columns: inverse along i1, x V, forward along i1
    for (int cc = grp; cc < N; cc += G) {
      cpx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int f = fof(r);
        v[r] = f >= 0 ? Y[f * N + rows_rot<N>(f, cc)] : cpx<T>{T(0), T(0)};
      }
      X::inverse(v, tw, l);
#pragma unroll
      for (int p = 0; p < R; ++p) v[p] = scale(v[p], V[(p + R * lq) * N + cc]);
      X::forward(v, tw, l);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int f = fof(r);
        if (f >= 0) Y[f * N + rows_rot<N>(f, cc)] = v[r];
      }
    }
    __syncthreads();
    // (C) rows, forward along i2, stick cells back
    for (int f = grp; f < nrow; f += G) {
      cpx<T>* yr = Y + f * N;
      cpx<T> v[R];
#pragma unroll
      for (int p = 0; p < R; ++p) v[p] = yr[rows_rot<N>(f, p + R * lq)];
      X::forward(v, tw, l);
#pragma unroll
      for (int r = 0; r < R; ++r) yr[rows_rot<N>(f, l + L * r)] = v[r];
      const int s1 = g.row_srange[2 * f + 1];
      for (int s = g.row_srange[2 * f] + l; s < s1; s += L) {
        const int i2 = g.stick_i12[s] % N;
        row[s] = yr[rows_rot<N>(f, i2)];
      }
    }
    // the next plane's (A) writes only rows this group owns; its (B) waits
    // for every group at the barrier after (A)
  }
}

// psi(r) planes of ncols vectors on the full grid
template <int N, int P, typename T>
__global__ __launch_bounds__((Strips<N, T>::NT)) void k_plane_to_grid_strips(
    GridDev g, VecSet<const cpx<T>> sticks, VecSet<cpx<T>> grid, const int* slots, int ncols,
    cpx<T>* scratch) {
  using S = Strips<N, T>;
  constexpr int NT = S::NT, CC = S::CC, CP = S::CP;
  extern __shared__ unsigned char smem_raw[];
  const StripLds<N, T> L(smem_raw, g);
  cpx<T>* Y = scratch + (long long)blockIdx.x * g.nrow * N;
  const long long nplanes = (long long)ncols * N;
  for (long long q = blockIdx.x; q < nplanes; q += gridDim.x) {
    const int c = int(q / N), i0 = int(q - (long long)c * N);
    const int slot = slots[c];
    const cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
    cpx<T>* dst = grid.base + slot * grid.stride + (long long)i0 * N * N;
    strips_rows_inverse<N, P, T>(L, g, row, Y);
    for (int c0 = 0; c0 < N; c0 += CC) {
      strips_cols_inverse<N, P, T>(L, Y, c0);
      for (int i = threadIdx.x; i < N * CC; i += NT) {
        const int i1 = i / CC, cc = i - i1 * CC;
        dst[i1 * N + c0 + cc] = L.tile[i1 * CP + cc];
      }
      __syncthreads();
    }
  }
}

// Delta n of perturbation j on plane i0 for every (j, i0) of the grid loop,
// summed over the bands in a fixed order (deterministic, no atomics)
template <int N, int P>
__global__ __launch_bounds__((Strips<N, double>::NT)) void k_drho_strips(
    GridDev g, const z64* sticks, long long sstride, int nband, const int* bands,
    const z64* psir, double coef, double* drho, int npert, z64* scratch) {
  using S = Strips<N, double>;
  constexpr int NT = S::NT, CC = S::CC, CP = S::CP, NCS = S::NCS;
  constexpr int PERS = (N * CC + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  const StripLds<N, double> L(smem_raw, g);
  z64* Y = scratch + (long long)blockIdx.x * g.nrow * N;
  const long long n3 = (long long)N * N * N;
  const long long nitems = (long long)npert * N;
  for (long long q = blockIdx.x; q < nitems; q += gridDim.x) {
    const int j = int(q / N), i0 = int(q - (long long)j * N);
    double acc[NCS][PERS];
#pragma unroll
    for (int cs = 0; cs < NCS; ++cs)
#pragma unroll
      for (int k = 0; k < PERS; ++k) acc[cs][k] = 0.0;
    for (int v = 0; v < nband; ++v) {
      const z64* row = sticks + ((long long)j * nband + v) * sstride + (long long)i0 * g.nst;
      strips_rows_inverse<N, P, double>(L, g, row, Y);
      const z64* pr = psir + (long long)bands[v] * n3 + (long long)i0 * N * N;
#pragma unroll
      for (int cs = 0; cs < NCS; ++cs) {
        strips_cols_inverse<N, P, double>(L, Y, cs * CC);
#pragma unroll
        for (int k = 0; k < PERS; ++k) {
          const int e = threadIdx.x + k * NT;
          if (e < N * CC) {
            const int i1 = e / CC, cc = e - i1 * CC;
            const z64 a = pr[i1 * N + cs * CC + cc], d = L.tile[i1 * CP + cc];
            acc[cs][k] += a.x * d.x + a.y * d.y;
          }
        }
        __syncthreads();
      }
    }
    double* out = drho + (long long)j * n3 + (long long)i0 * N * N;
#pragma unroll
    for (int cs = 0; cs < NCS; ++cs)
#pragma unroll
      for (int k = 0; k < PERS; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < N * CC) {
          const int i1 = e / CC, cc = e - i1 * CC;
          out[i1 * N + cs * CC + cc] = coef * acc[cs][k];
        }
      }
  }
}

// Raises the dynamic LDS limit of one kernel instantiation once per process.
template <auto K>
void set_smem(size_t bytes) {
  static bool done = false;
  if (!done) {
    STH_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(K),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
  }
}

template <typename T>
int plan_of(const GridDev& g) { return g.plan[sizeof(T) == 4 ? 1 : 0]; }

}  // namespace

// Compile-time dispatch over (grid length, radix plan).
#define STH_DISPATCH_NP(Nval, Pval, ...)                                              \
  do {                                                                                \
    const int _p = (Pval);                                                            \
    switch (Nval * 4 + _p) {                                                          \
      case 24 * 4 + 0: { constexpr int NN = 24, PP = 0; __VA_ARGS__; } break;        \
      case 24 * 4 + 1: { constexpr int NN = 24, PP = 1; __VA_ARGS__; } break;        \
      case 48 * 4 + 0: { constexpr int NN = 48, PP = 0; __VA_ARGS__; } break;        \
      case 48 * 4 + 1: { constexpr int NN = 48, PP = 1; __VA_ARGS__; } break;        \
      case 72 * 4 + 0: { constexpr int NN = 72, PP = 0; __VA_ARGS__; } break;        \
      case 72 * 4 + 1: { constexpr int NN = 72, PP = 1; __VA_ARGS__; } break;        \
      case 96 * 4 + 0: { constexpr int NN = 96, PP = 0; __VA_ARGS__; } break;        \
      case 96 * 4 + 1: { constexpr int NN = 96, PP = 1; __VA_ARGS__; } break;        \
      default:                                                                        \
        set_error("unsupported FFT grid %d / plan %d (grids 24, 48, 72, 96)", Nval, _p); \
        throw Error(STH_E_INVALID);                                                   \
    }                                                                                 \
  } while (0)

// Every grid, including those whose plane tile exceeds the LDS (z-stick and
// strip-form kernels).
#define STH_DISPATCH_ALL(Nval, Pval, ...)                                             \
  do {                                                                                \
    if ((Nval) == 144) {                                                              \
      switch (Pval) {                                                                 \
        case 0: { constexpr int NN = 144, PP = 0; __VA_ARGS__; } break;              \
        case 1: { constexpr int NN = 144, PP = 1; __VA_ARGS__; } break;              \
        default:                                                                      \
          set_error("unsupported radix plan %d for grid 144", (Pval));                \
          throw Error(STH_E_INVALID);                                                 \
      }                                                                               \
    } else {                                                                          \
      STH_DISPATCH_NP(Nval, Pval, __VA_ARGS__);                                       \
    }                                                                                 \
  } while (0)

// The strip form runs where the tile does not fit, or where it was chosen.
inline bool use_strips(const GridDev& g, int kind) {
  return g.N > kTileMaxN || kind == kPlaneStrips;
}

inline void check_stage(const GridDev& g) {
  if (!g.stage || g.stage_slots <= 0) {
    set_error("internal: strip-form plane kernel without scratch planes");
    throw Error(STH_E_INTERNAL);
  }
}

// z-stick kernel form (GridDev::zfft_kind): 0 workgroup form, 1 wave form.
template <typename T, typename Tin>
void launch_zfft_inv(const GridDev& g, VecSet<const Tin> in, VecSet<cpx<T>> sticks,
                     const int* slots, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  const int kind = g.zfft_kind[sizeof(T) == 4 ? 1 : 0];
  STH_DISPATCH_ALL(g.N, plan_of<T>(g), {
    if (kind == 0) {
      constexpr int ZS = zsticks<NN, T>();
      dim3 grid((g.nst + ZS - 1) / ZS, ncols);
      hipLaunchKernelGGL((k_zfft_inv<NN, PP, T, Tin>), grid, dim3(zthreads<NN, PP, T>()), 0, st,
                         g, in, sticks, slots);
    } else {
      using Z = ZWave<NN, PP, T>;
      dim3 grid((g.nst + Z::ZS - 1) / Z::ZS, ncols);
      hipLaunchKernelGGL((k_zfft_inv_wave<NN, PP, T, Tin>), grid, dim3(Z::NT), 0, st, g, in,
                         sticks, slots);
    }
  });
  STH_HIP_CHECK(hipGetLastError());
}

// Compute units of the current device (the persistent plane form sizes its
// grid by them).
inline int device_cus() {
  static const int n = [] {
    int dev = 0, v = 0;
    STH_HIP_CHECK(hipGetDevice(&dev));
    STH_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
    return v > 0 ? v : 1;
  }();
  return n;
}

// Largest dynamic LDS of one workgroup on the current device.
inline size_t device_max_lds() {
  static const size_t n = [] {
    int dev = 0, v = 0;
    STH_HIP_CHECK(hipGetDevice(&dev));
    STH_HIP_CHECK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    return size_t(v > 0 ? v : 65536);
  }();
  return n;
}

template <int N, typename T>
void launch_plane_rows(const GridDev& g, VecSet<cpx<T>> sticks, const int* slots, int ncols,
                       const T* pot, const T* const* pot_ptr, hipStream_t st) {
  const size_t sm = rows_lds_bytes<N, T>(g.nrow);
  if (sm > device_max_lds() || !g.row_srange) {
    set_error("compact-row plane kernel: %d rows of %d need %zu B of LDS (%zu available)",
              g.nrow, N, sm, device_max_lds());
    throw Error(STH_E_INVALID);
  }
  static std::mutex mu;
  static std::map<size_t, int> per_cu_of;
  int per_cu;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = per_cu_of.find(sm);
    if (it == per_cu_of.end()) {
      int b = 0;
      STH_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &b, reinterpret_cast<const void*>(&k_plane_rows<N, T>), RowsForm<N, T>::NT, sm));
      it = per_cu_of.emplace(sm, b > 0 ? b : 1).first;
    }
    per_cu = it->second;
  }
  const long long np = (long long)ncols * N;
  const dim3 pg((unsigned)std::min<long long>(np, (long long)per_cu * device_cus()));
  hipLaunchKernelGGL((k_plane_rows<N, T>), pg, dim3(RowsForm<N, T>::NT), sm, st, g, sticks, slots,
                     ncols, pot, pot_ptr);
}

bool plane_kind_available(const GridDev& g, int kind, bool fp32) {
  if (kind < 0 || kind >= kPlaneKinds) return false;
  if (kind == kPlaneStrips) return true;
  if (kind == kPlaneRows) {
    if (!g.row_srange) return false;
    size_t sm = 0;
    STH_DISPATCH_ALL(g.N, 0, {
      sm = fp32 ? rows_lds_bytes<NN, float>(g.nrow) : rows_lds_bytes<NN, double>(g.nrow);
    });
    return sm <= device_max_lds();
  }
  return g.N <= kTileMaxN;
}

// Plane kernel variants (GridDev::plane_kind): 0 single-pass workgroup form,
// 1 wave form, 2 strip form (the only tile-free form besides 4), 3 persistent
// single-pass form with the next plane's loads in flight, 4 compact-row form.
template <typename T>
void launch_plane_local(const GridDev& g, VecSet<cpx<T>> sticks, const int* slots, int ncols,
                        const T* pot, const T* const* pot_ptr, hipStream_t st) {
  if (ncols <= 0) return;
  dim3 grid(g.N, ncols);
  const int kind = g.plane_kind[sizeof(T) == 4 ? 1 : 0];
  if (kind == kPlaneRows) {
    STH_DISPATCH_ALL(g.N, 0, {
      launch_plane_rows<NN, T>(g, sticks, slots, ncols, pot, pot_ptr, st);
    });
    STH_HIP_CHECK(hipGetLastError());
    return;
  }
  if (use_strips(g, kind)) {
    check_stage(g);
    STH_DISPATCH_ALL(g.N, plan_of<T>(g), {
      using S = Strips<NN, T>;
      const long long np = (long long)ncols * NN;
      const dim3 sg((unsigned)std::min<long long>(np, g.stage_slots));
      hipLaunchKernelGGL((k_plane_strips<NN, PP, T>), sg, dim3(S::NT), S::lds_bytes, st, g,
                         sticks, slots, ncols, pot, pot_ptr, static_cast<cpx<T>*>(g.stage));
    });
    STH_HIP_CHECK(hipGetLastError());
    return;
  }
  if (2 * g.nrow > g.N) {   // an alias-free sphere has at most N/2 rows
    set_error("plane kernel: %d active rows exceed N/2 = %d", g.nrow, g.N / 2);
    throw Error(STH_E_INVALID);
  }
  STH_DISPATCH_NP(g.N, plan_of<T>(g), {
    if (kind == 0) {
      constexpr size_t sm = fused_lds_bytes<NN, T>();
      constexpr int nt = fused_threads<NN, PP>();
      hipLaunchKernelGGL((k_plane_fused<NN, PP, T>), grid, dim3(nt), sm, st, g, sticks, slots,
                         pot, pot_ptr);
    } else if (kind == kPlanePersistent) {
      constexpr size_t sm = pf_lds_bytes<NN, T>();
      constexpr int nt = fused_threads<NN, PP>();
      if (g.nst > pf_sticks_per_thread<NN, PP>() * nt) {
        set_error("persistent plane kernel: %d sticks exceed %d", g.nst,
                  pf_sticks_per_thread<NN, PP>() * nt);
        throw Error(STH_E_INVALID);
      }
      static const int per_cu = [] {
        int b = 0;
        STH_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &b, reinterpret_cast<const void*>(&k_plane_fused_pf<NN, PP, T>), nt, sm));
        return b > 0 ? b : 1;
      }();
      const long long np = (long long)ncols * NN;
      const dim3 pg((unsigned)std::min<long long>(np, (long long)per_cu * device_cus()));
      hipLaunchKernelGGL((k_plane_fused_pf<NN, PP, T>), pg, dim3(nt), sm, st, g, sticks, slots,
                         ncols, pot, pot_ptr);
    } else {
      using S = PlaneWave<NN, PP>;
      constexpr size_t sm = S::lds_bytes(sizeof(cpx<T>));
      hipLaunchKernelGGL((k_plane_wave<NN, PP, T>), grid, dim3(S::NT), sm, st, g, sticks, slots,
                         pot, pot_ptr);
    }
  });
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T, typename Tout>
void launch_zfft_fwd(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<Tout> out,
                     const int* slots, int ncols, int mode, VecSet<const Tout> pin,
                     const double* eps_slot, hipStream_t st) {
  if (ncols <= 0) return;
  const int kind = g.zfft_kind[sizeof(T) == 4 ? 1 : 0];
  STH_DISPATCH_ALL(g.N, plan_of<T>(g), {
    if (kind == 0) {
      constexpr int ZS = zsticks<NN, T>();
      dim3 grid((g.nst + ZS - 1) / ZS, ncols);
      hipLaunchKernelGGL((k_zfft_fwd<NN, PP, T, Tout>), grid, dim3(zthreads<NN, PP, T>()), 0, st,
                         g, sticks, out, slots, mode, pin, eps_slot);
    } else {
      using Z = ZWave<NN, PP, T>;
      dim3 grid((g.nst + Z::ZS - 1) / Z::ZS, ncols);
      hipLaunchKernelGGL((k_zfft_fwd_wave<NN, PP, T, Tout>), grid, dim3(Z::NT), 0, st, g, sticks,
                         out, slots, mode, pin, eps_slot);
    }
  });
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_plane_to_grid(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<cpx<T>> grid_out,
                          const int* slots, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  if (use_strips(g, g.plane_kind[sizeof(T) == 4 ? 1 : 0])) {
    check_stage(g);
    STH_DISPATCH_ALL(g.N, plan_of<T>(g), {
      using S = Strips<NN, T>;
      const long long np = (long long)ncols * NN;
      const dim3 sg((unsigned)std::min<long long>(np, g.stage_slots));
      hipLaunchKernelGGL((k_plane_to_grid_strips<NN, PP, T>), sg, dim3(S::NT), S::lds_bytes, st,
                         g, sticks, grid_out, slots, ncols, static_cast<cpx<T>*>(g.stage));
    });
    STH_HIP_CHECK(hipGetLastError());
    return;
  }
  dim3 grid(g.N, ncols);
  STH_DISPATCH_NP(g.N, plan_of<T>(g), {
    constexpr size_t sm = PlaneLds<NN, T>::bytes(false);
    set_smem<k_plane_to_grid<NN, PP, T>>(sm);
    hipLaunchKernelGGL((k_plane_to_grid<NN, PP, T>), grid, dim3(pthreads<NN, PP>()), sm, st, g,
                       sticks, grid_out, slots);
  });
  STH_HIP_CHECK(hipGetLastError());
}

void launch_drho(const GridDev& g, const z64* sticks, long long stick_stride, int nband,
                 const int* bands, const z64* psir, int npert, double coef, double* drho,
                 hipStream_t st) {
  if (npert <= 0) return;
  if (use_strips(g, g.plane_kind[0])) {
    check_stage(g);
    STH_DISPATCH_ALL(g.N, plan_of<double>(g), {
      using S = Strips<NN, double>;
      const long long ni = (long long)npert * NN;
      const dim3 sg((unsigned)std::min<long long>(ni, g.stage_slots));
      hipLaunchKernelGGL((k_drho_strips<NN, PP>), sg, dim3(S::NT), S::lds_bytes, st, g, sticks,
                         stick_stride, nband, bands, psir, coef, drho, npert,
                         static_cast<z64*>(g.stage));
    });
    STH_HIP_CHECK(hipGetLastError());
    return;
  }
  dim3 grid(g.N, npert);
  STH_DISPATCH_NP(g.N, plan_of<double>(g), {
    constexpr size_t sm = PlaneLds<NN, double>::bytes(false);
    set_smem<k_drho<NN, PP>>(sm);
    hipLaunchKernelGGL((k_drho<NN, PP>), grid, dim3(pthreads<NN, PP>()), sm, st, g, sticks,
                       stick_stride, nband, bands, psir, coef, drho);
  });
  STH_HIP_CHECK(hipGetLastError());
}

// Sets the LDS limits of every plane kernel of grid N up front, so that no
// attribute call happens while a stream is being captured into a graph.
void prepare_fft_kernels(int N) {
  STH_DISPATCH_ALL(N, 0, {
    set_smem<k_plane_rows<NN, double>>(device_max_lds());
    set_smem<k_plane_rows<NN, float>>(device_max_lds());
  });
  for (int p = 0; p < kRadixPlans; ++p) {
    STH_DISPATCH_ALL(N, p, {
      set_smem<k_plane_strips<NN, PP, double>>(Strips<NN, double>::lds_bytes);
      set_smem<k_plane_strips<NN, PP, float>>(Strips<NN, float>::lds_bytes);
      set_smem<k_plane_to_grid_strips<NN, PP, double>>(Strips<NN, double>::lds_bytes);
      set_smem<k_drho_strips<NN, PP>>(Strips<NN, double>::lds_bytes);
    });
    if (N > kTileMaxN) continue;
    STH_DISPATCH_NP(N, p, {
      set_smem<k_plane_fused<NN, PP, double>>(fused_lds_bytes<NN, double>());
      set_smem<k_plane_fused<NN, PP, float>>(fused_lds_bytes<NN, float>());
      set_smem<k_plane_fused_pf<NN, PP, double>>(pf_lds_bytes<NN, double>());
      set_smem<k_plane_fused_pf<NN, PP, float>>(pf_lds_bytes<NN, float>());
      set_smem<k_plane_wave<NN, PP, double>>(PlaneWave<NN, PP>::lds_bytes(sizeof(z64)));
      set_smem<k_plane_wave<NN, PP, float>>(PlaneWave<NN, PP>::lds_bytes(sizeof(z32)));
      set_smem<k_plane_to_grid<NN, PP, double>>(PlaneLds<NN, double>::bytes(false));
      set_smem<k_drho<NN, PP>>(PlaneLds<NN, double>::bytes(false));
    });
  }
}

template void launch_zfft_inv<double, z64>(const GridDev&, VecSet<const z64>, VecSet<z64>,
                                           const int*, int, hipStream_t);
template void launch_zfft_inv<float, z64>(const GridDev&, VecSet<const z64>, VecSet<z32>,
                                          const int*, int, hipStream_t);
template void launch_plane_local<double>(const GridDev&, VecSet<z64>, const int*, int,
                                         const double*, const double* const*, hipStream_t);
template void launch_plane_local<float>(const GridDev&, VecSet<z32>, const int*, int,
                                        const float*, const float* const*, hipStream_t);
template void launch_zfft_fwd<double, z64>(const GridDev&, VecSet<const z64>, VecSet<z64>,
                                           const int*, int, int, VecSet<const z64>,
                                           const double*, hipStream_t);
template void launch_zfft_fwd<float, z64>(const GridDev&, VecSet<const z32>, VecSet<z64>,
                                          const int*, int, int, VecSet<const z64>,
                                          const double*, hipStream_t);
template void launch_plane_to_grid<double>(const GridDev&, VecSet<const z64>, VecSet<z64>,
                                           const int*, int, hipStream_t);

}  // namespace sth
