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
//              are scattered into an N x N LDS tile, inverse-transformed along
//              i2 (only rows that hold sticks) and i1, multiplied by the real
//              potential (fused into the stores of the last inverse pass),
//              transformed forward and gathered back.
//   zfft_fwd   z-sticks -> sphere: forward transform along axis 0, 1/N^3, the
//              sphere components extracted, kinetic and shift terms fused.
// Every kernel is instantiated for each radix plan of its length; the plan used
// is chosen per system and precision (GridDev::plan, set by the autotuner).
// Workgroups have as many threads as the widest pass has butterflies, so each
// pass is one round of work between two barriers.
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
  return (64 * (N + 1) * int(sizeof(cpx<T>)) > 40960) ? 32 : 64;
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

template <int N, int P, typename T>
__global__ __launch_bounds__((pthreads<N, P>())) void k_plane_local(GridDev g,
                                                                   VecSet<cpx<T>> sticks,
                                                                   const int* slots, const T* pot,
                                                                   const T* const* pot_ptr) {
  constexpr int NT = pthreads<N, P>();
  constexpr int NP = N + 1;
  extern __shared__ unsigned char smem_raw[];
  PlaneLds<N, T> L(smem_raw);
  const int slot = slots[blockIdx.y];
  const int i0 = blockIdx.x;
  cpx<T>* row = sticks.base + slot * sticks.stride + (long long)i0 * g.nst;
  const T* V = (pot_ptr ? pot_ptr[slot] : pot) + (long long)i0 * N * N;
  plane_stage<N, NT, T>(L, g);
  if constexpr (PlaneLds<N, T>::kStageV) {
    for (int e = threadIdx.x; e < N * N; e += NT) L.v[e] = V[e];   // coalesced
  }
  plane_scatter<N, NT, T>(L, g, row);
  if constexpr (PlaneLds<N, T>::kStageV) {
    const T* lv = L.v;
    plane_inverse<N, P, NT, T>(L, g, [lv](int a, cpx<T> c) {
      const int i1 = a / NP, i2 = a - (a / NP) * NP;
      const T s = lv[i1 * N + i2];
      return cpx<T>{c.x * s, c.y * s};
    });
  } else {
    plane_inverse<N, P, NT, T>(L, g);
    for (int e = threadIdx.x; e < N * N; e += NT) {
      const int i1 = e / N, i2 = e - (e / N) * N;
      const T s = V[e];
      cpx<T>& c = L.pl[i1 * NP + i2];
      c.x *= s;
      c.y *= s;
    }
    __syncthreads();
  }
  plane_forward<N, P, NT, T>(L, g);
  for (int s = threadIdx.x; s < g.nst; s += NT) {
    const int p = g.stick_i12[s];
    const int i1 = p / N, i2 = p - (p / N) * N;
    row[s] = L.pl[i1 * NP + i2];
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

template <typename T, typename Tin>
void launch_zfft_inv(const GridDev& g, VecSet<const Tin> in, VecSet<cpx<T>> sticks,
                     const int* slots, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  STH_DISPATCH_NP(g.N, plan_of<T>(g), {
    constexpr int ZS = zsticks<NN, T>();
    dim3 grid((g.nst + ZS - 1) / ZS, ncols);
    hipLaunchKernelGGL((k_zfft_inv<NN, PP, T, Tin>), grid, dim3(zthreads<NN, PP, T>()), 0, st,
                       g, in, sticks, slots);
  });
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_plane_local(const GridDev& g, VecSet<cpx<T>> sticks, const int* slots, int ncols,
                        const T* pot, const T* const* pot_ptr, hipStream_t st) {
  if (ncols <= 0) return;
  dim3 grid(g.N, ncols);
  STH_DISPATCH_NP(g.N, plan_of<T>(g), {
    constexpr size_t sm = PlaneLds<NN, T>::bytes(true);
    set_smem<k_plane_local<NN, PP, T>>(sm);
    hipLaunchKernelGGL((k_plane_local<NN, PP, T>), grid, dim3(pthreads<NN, PP>()), sm, st, g,
                       sticks, slots, pot, pot_ptr);
  });
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T, typename Tout>
void launch_zfft_fwd(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<Tout> out,
                     const int* slots, int ncols, int mode, VecSet<const Tout> pin,
                     const double* eps_slot, hipStream_t st) {
  if (ncols <= 0) return;
  STH_DISPATCH_NP(g.N, plan_of<T>(g), {
    constexpr int ZS = zsticks<NN, T>();
    dim3 grid((g.nst + ZS - 1) / ZS, ncols);
    hipLaunchKernelGGL((k_zfft_fwd<NN, PP, T, Tout>), grid, dim3(zthreads<NN, PP, T>()), 0, st,
                       g, sticks, out, slots, mode, pin, eps_slot);
  });
  STH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_plane_to_grid(const GridDev& g, VecSet<const cpx<T>> sticks, VecSet<cpx<T>> grid_out,
                          const int* slots, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
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
  for (int p = 0; p < kRadixPlans; ++p) {
    STH_DISPATCH_NP(N, p, {
      set_smem<k_plane_local<NN, PP, double>>(PlaneLds<NN, double>::bytes(true));
      set_smem<k_plane_local<NN, PP, float>>(PlaneLds<NN, float>::bytes(true));
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
