// Shared device/host helpers of the Sternheimer library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sth {

// Interleaved complex number (re, im) of real type T.  8- or 16-byte aligned so a
// single global load moves the whole value.
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};
using z64 = cpx<double>;
using z32 = cpx<float>;

template <typename T>
__host__ __device__ inline cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T>
__host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ inline cpx<T> scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__host__ __device__ inline cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse):  SIGN = -1 gives -i * a
template <int SIGN, typename T>
__host__ __device__ inline cpx<T> mul_i(cpx<T> a) {
  return SIGN < 0 ? cpx<T>{a.y, -a.x} : cpx<T>{-a.y, a.x};
}

// Workgroups are dispatched to the chip's 8 XCDs round-robin by linear id, and
// each XCD has its own L2 (the 256 MB last-level cache is shared).  xcd_tile2
// maps the workgroups of one (x, y) slice of the grid so that every XCD gets
// one contiguous range of logical tiles, x fastest (or y fastest): tiles that
// share an operand along the fast index run on one XCD, one after the other,
// while z (the K-chunk of a split-K product) stays the slowest index of the
// dispatch order, so that all XCDs work on the same chunk at a time.  A
// bijection of each slice for any size.
__device__ inline void xcd_tile2(bool yfast, int& x, int& y) {
  const long long gx = gridDim.x, gy = gridDim.y;
  const long long S = gx * gy;
  const long long L = blockIdx.x + gx * (long long)blockIdx.y;
  const long long q = S / 8, r = S % 8, xcd = L % 8, j = L / 8;
  const long long lg = xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
  if (yfast) {
    y = int(lg % gy);
    x = int(lg / gy);
  } else {
    x = int(lg % gx);
    y = int(lg / gx);
  }
}

}  // namespace sth

#define STH_HIP_CHECK(expr)                                                      \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) {                                                      \
      ::sth::set_error("HIP error %s at %s:%d: %s", hipGetErrorString(_e),      \
                       __FILE__, __LINE__, #expr);                               \
      throw ::sth::Error(STH_E_DEVICE);                                          \
    }                                                                            \
  } while (0)
