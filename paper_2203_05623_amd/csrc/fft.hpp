// Mixed-radix FFT building blocks for gfx950 (HIP).
//
// Small DFT codelets (radix 2, 3, 4, 6, 8, 9, 16) and a self-sorting
// (Stockham) pass that runs many short FFTs held in LDS by one workgroup.
// All FFT lengths of the workloads are 2^a 3^b (24, 48, 72, 96, 144).
//
// Stockham pass with radix R after a product NS of earlier radices: the
// butterfly j in [0, N/R) reads x[j + r N/R], r < R, multiplies element r by
// w_N^(r (j mod NS) N/(NS R)), takes the length-R DFT and writes element r to
// ((j / NS) NS R + j mod NS) + r NS.  Chaining the passes of any
// factorisation N = R1 R2 ... leaves the result in natural order.
//
// SIGN = -1 is the forward transform exp(-2 pi i jk/N), SIGN = +1 the inverse
// (both unnormalised).  Twiddles come from a table tw[t] = exp(-2 pi i t / N)
// computed in FP64 on the host (conjugated here for the inverse).
#pragma once

#include "common.hpp"

namespace sth {

// ------------------------------------------------------------------ codelets
template <int SIGN, typename T>
__host__ __device__ inline void dft2(cpx<T>& a, cpx<T>& b) {
  cpx<T> t = a;
  a = t + b;
  b = t - b;
}

template <int SIGN, typename T>
__host__ __device__ inline void dft3(cpx<T>& a, cpx<T>& b, cpx<T>& c) {
  const T s3 = T(0.86602540378443864676);  // sqrt(3)/2
  cpx<T> t1 = b + c;
  cpx<T> t2 = a - scale(t1, T(0.5));
  cpx<T> t3 = mul_i<SIGN>(scale(b - c, s3));
  a = a + t1;
  b = t2 + t3;
  c = t2 - t3;
}

template <int SIGN, typename T>
__host__ __device__ inline void dft4(cpx<T>& a, cpx<T>& b, cpx<T>& c, cpx<T>& d) {
  cpx<T> t0 = a + c, t1 = a - c, t2 = b + d, t3 = mul_i<SIGN>(b - d);
  a = t0 + t2;
  c = t0 - t2;
  b = t1 + t3;
  d = t1 - t3;
}

template <int R, int SIGN, typename T>
struct Dft;

template <int SIGN, typename T>
struct Dft<2, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft2<SIGN>(v[0], v[1]); }
};
template <int SIGN, typename T>
struct Dft<3, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft3<SIGN>(v[0], v[1], v[2]); }
};
template <int SIGN, typename T>
struct Dft<4, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft4<SIGN>(v[0], v[1], v[2], v[3]); }
};

// radix 8: two radix-4 halves (even / odd samples) joined by w8^k
template <int SIGN, typename T>
struct Dft<8, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) {
    const T h = T(0.70710678118654752440);
    cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<SIGN>(e0, e1, e2, e3);
    dft4<SIGN>(o0, o1, o2, o3);
    // w8^1 = h (1 + SIGN i), w8^2 = SIGN i, w8^3 = h (-1 + SIGN i)
    cpx<T> w1o1 = scale(o1 + mul_i<SIGN>(o1), h);
    cpx<T> w2o2 = mul_i<SIGN>(o2);
    cpx<T> w3o3 = scale(mul_i<SIGN>(o3) - o3, h);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + w1o1;
    v[5] = e1 - w1o1;
    v[2] = e2 + w2o2;
    v[6] = e2 - w2o2;
    v[3] = e3 + w3o3;
    v[7] = e3 - w3o3;
  }
};

// Composite codelet R = P * Q:  n = P n1 + n2 (n1 < Q, n2 < P), k = k1 + Q k2.
// Inner DFTs of length Q over n1, twiddle w_R^(n2 k1), outer DFTs of length P over
// n2.  Both stages work in place on v (an inner DFT reads and writes the cells
// P n1 + n2 of one n2, an outer DFT the cells P k1 + n2 of one k1), so at most
// R + max(P, Q) values are live; the final reordering is a register renaming.
template <int P, int Q, int SIGN, typename T>
__host__ __device__ inline void dft_composite(cpx<T>* v) {
  constexpr int R = P * Q;
#pragma unroll
  for (int n2 = 0; n2 < P; ++n2) {
    cpx<T> t[Q];
#pragma unroll
    for (int n1 = 0; n1 < Q; ++n1) t[n1] = v[P * n1 + n2];
    Dft<Q, SIGN, T>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) {
      if (n2 * k1 == 0) {
        v[P * k1 + n2] = t[k1];
      } else {
        // exp(SIGN 2 pi i n2 k1 / R), folded to constants by the compiler
        const double ang = 6.283185307179586476925 * double(n2 * k1) / double(R);
        const cpx<T> w = {T(__builtin_cos(ang)), T(SIGN * __builtin_sin(ang))};
        v[P * k1 + n2] = t[k1] * w;
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < Q; ++k1) {
    cpx<T> t[P];
#pragma unroll
    for (int n2 = 0; n2 < P; ++n2) t[n2] = v[P * k1 + n2];
    Dft<P, SIGN, T>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < P; ++k2) v[P * k1 + k2] = t[k2];
  }
  // v[P k1 + k2] holds X[k1 + Q k2]
  cpx<T> o[R];
#pragma unroll
  for (int k1 = 0; k1 < Q; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < P; ++k2) o[k1 + Q * k2] = v[P * k1 + k2];
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = o[i];
}

template <int SIGN, typename T>
struct Dft<6, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft_composite<2, 3, SIGN, T>(v); }
};
template <int SIGN, typename T>
struct Dft<9, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft_composite<3, 3, SIGN, T>(v); }
};
template <int SIGN, typename T>
struct Dft<16, SIGN, T> {
  __host__ __device__ static void run(cpx<T>* v) { dft_composite<4, 4, SIGN, T>(v); }
};

// ------------------------------------------------------------------ LDS passes
// Butterfly task t of a pass over nfft transforms: transform f = t / (N/R),
// butterfly j = t mod (N/R).  base(f) gives the LDS offset of element 0 of
// transform f and ES the element stride.
template <typename T, int N, int R, int NS, int SIGN>
__host__ __device__ inline void stockham_load(const cpx<T>* buf, int base, int es, int j,
                                              cpx<T>* v) {
  constexpr int M = N / R;
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[base + (j + r * M) * es];
}

// Output hook of the last pass: identity (store the transform as is).
struct NoPost {
  template <typename C>
  __host__ __device__ C operator()(int, C v) const { return v; }
};

template <typename T, int N, int R, int NS, int SIGN, typename Post = NoPost>
__host__ __device__ inline void stockham_compute_store(cpx<T>* buf, int base, int es, int j,
                                                       cpx<T>* v, const cpx<T>* tw,
                                                       Post post = Post()) {
  constexpr int STEP = N / (NS * R);
  const int k = j % NS;
  if (NS > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cpx<T> w = tw[r * k * STEP];
      if (SIGN > 0) w.y = -w.y;
      v[r] = v[r] * w;
    }
  }
  Dft<R, SIGN, T>::run(v);
  const int d = (j / NS) * NS * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int a = base + (d + r * NS) * es;
    buf[a] = post(a, v[r]);
  }
}

// One in-place pass over nfft transforms by the whole workgroup (NTHR threads).
// All butterflies are loaded to registers before the barrier and stored after
// it, so the pass can work in place.
template <typename T, int N, int R, int NS, int SIGN, int NTHR, int NFFTMAX, typename BaseFn,
          typename Post = NoPost>
__device__ inline void lds_pass(cpx<T>* buf, int nfft, int es, BaseFn base_of, const cpx<T>* tw,
                                Post post = Post()) {
  constexpr int M = N / R;
  constexpr int MAXT = (NFFTMAX * M + NTHR - 1) / NTHR;
  const int ntask = nfft * M;
  cpx<T> v[MAXT][R];
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = threadIdx.x + q * NTHR;
    if (t < ntask) {
      const int f = t / M, j = t - f * M;
      stockham_load<T, N, R, NS, SIGN>(buf, base_of(f), es, j, v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = threadIdx.x + q * NTHR;
    if (t < ntask) {
      const int f = t / M, j = t - f * M;
      stockham_compute_store<T, N, R, NS, SIGN>(buf, base_of(f), es, j, v[q], tw, post);
    }
  }
  __syncthreads();
}

// A full length-N transform as a chain of passes with radices R0, RS...; `post`
// maps every output value (with its LDS index) as the last pass stores it.
template <typename T, int N, int SIGN, int NTHR, int NFFTMAX, int NS, int R0, int... RS>
struct LdsFFT {
  template <typename BaseFn, typename Post = NoPost>
  __device__ static void run(cpx<T>* buf, int nfft, int es, BaseFn base_of, const cpx<T>* tw,
                             Post post = Post()) {
    if constexpr (sizeof...(RS) > 0) {
      lds_pass<T, N, R0, NS, SIGN, NTHR, NFFTMAX>(buf, nfft, es, base_of, tw);
      LdsFFT<T, N, SIGN, NTHR, NFFTMAX, NS * R0, RS...>::run(buf, nfft, es, base_of, tw, post);
    } else {
      lds_pass<T, N, R0, NS, SIGN, NTHR, NFFTMAX>(buf, nfft, es, base_of, tw, post);
    }
  }
};

// Threads that make every pass of a radix plan a single round over nfft
// transforms (one butterfly per thread), rounded to whole wavefronts, at most 1024.
template <int N, int R0, int... RS>
constexpr int pass_threads(int nfft) {
  int rmin = R0;
  ((rmin = RS < rmin ? RS : rmin), ...);
  const int t = nfft * (N / rmin);
  const int w = ((t + 63) / 64) * 64;
  return w > 1024 ? 1024 : w;
}

// Radix plans per length (first radix applied first); two plans per length,
// chosen per system and precision by the autotuner (plan 0 is the default).
template <int N, int P>
struct RadixPlan;
#define STH_RADIX_PLAN(NV, PV, ...)                                             \
  template <>                                                                   \
  struct RadixPlan<NV, PV> {                                                    \
    template <typename T, int SIGN, int NTHR, int NFFTMAX>                      \
    using fft = LdsFFT<T, NV, SIGN, NTHR, NFFTMAX, 1, __VA_ARGS__>;             \
    static constexpr int threads(int nfft) { return pass_threads<NV, __VA_ARGS__>(nfft); } \
    static constexpr int radix(int i) {                                         \
      constexpr int rs[] = {__VA_ARGS__};                                       \
      return rs[i];                                                             \
    }                                                                           \
  };
STH_RADIX_PLAN(24, 0, 8, 3)
STH_RADIX_PLAN(24, 1, 4, 6)
STH_RADIX_PLAN(48, 0, 16, 3)
STH_RADIX_PLAN(48, 1, 8, 6)
STH_RADIX_PLAN(72, 0, 8, 9)
STH_RADIX_PLAN(72, 1, 9, 8)
STH_RADIX_PLAN(96, 0, 16, 6)
STH_RADIX_PLAN(96, 1, 6, 16)
STH_RADIX_PLAN(144, 0, 16, 9)
STH_RADIX_PLAN(144, 1, 9, 16)
#undef STH_RADIX_PLAN
constexpr int kRadixPlans = 2;

// ------------------------------------------------------------------ two-pass plans
// Every plan above has two radices, N = R1 R2.  The inverse transform is pass 1
// (radix R1, N/R1 butterflies, no twiddles) then pass 2 (radix R2, N/R2 = R1
// butterflies; butterfly j reads and writes the cells j + r R1 and multiplies
// input r by exp(+2 pi i r j / N)).  The forward transform is used in the form
// of the adjoint of that sequence: pass 2^H (DFT of sign -1 over the cells
// j + q R1, then the conjugate twiddles, written back to the same cells) and
// pass 1^H (reads the cells where pass 1 wrote, writes natural order).
//
// w[r] = exp(+2 pi i r j / N), r < R, from w1 = tw[j] = exp(-2 pi i j / N) by a
// balanced product tree (each power is at most ceil(log2 R) products deep).
template <int R, typename T>
__host__ __device__ inline void twiddle_powers(cpx<T> w1, cpx<T>* w) {
  w1.y = -w1.y;
  w[0] = cpx<T>{T(1), T(0)};
  if constexpr (R > 1) w[1] = w1;
#pragma unroll
  for (int r = 2; r < R; ++r) w[r] = w[r / 2] * w[r - r / 2];
}

}  // namespace sth
