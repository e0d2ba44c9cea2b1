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
// each XCD has its own L2.  The logical tile (x, y, z) of a workgroup is taken
// so that every XCD gets one contiguous range of logical ids in x-fastest
// order: tiles that share an operand along x run on one XCD, one after the
// other.  A bijection of the grid for any size.
__device__ inline void xcd_tile3(int& x, int& y, int& z) {
  const long long gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const long long T = gx * gy * gz;
  const long long L = blockIdx.x + gx * (blockIdx.y + gy * (long long)blockIdx.z);
  const long long q = T / 8, r = T % 8, xcd = L % 8, j = L / 8;
  const long long lg = xcd < r ? xcd * (q + 1) + j : r * (q + 1) + (xcd - r) * q + j;
  x = int(lg % gx);
  y = int((lg / gx) % gy);
  z = int(lg / (gx * gy));
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
