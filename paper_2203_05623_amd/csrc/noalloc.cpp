// H c for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the variant
// of sth_apply_h whose work space (vectors in internal order, z-stick scratch,
// split-K partials of the projector GEMM, column lists) is one file-scope
// device array of kNoAllocBytes per GPU, held until the process ends.
//
// The array's name is a host-side stand-in in host code; its device address is
// taken once per device (hipGetSymbolAddress, with that device current) when a
// context is created, and only that address reaches the kernels.  Every call
// on a GPU shares the array: calls that overlap on one GPU race, and the
// contents are those of the last call (the column lists and zero shifts are
// rewritten by a fill kernel on every call).
#include <map>
#include <mutex>

#include "engine.hpp"

namespace sth {

namespace {

constexpr size_t kNoAllocBytes = size_t(64) << 20;   // 64 MiB per GPU

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
std::map<int, unsigned char*> g_scratch;   // device ordinal -> device address of `scratch`

__global__ void k_fill_lists(int* ids, double* zeros, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    ids[i] = i;
    zeros[i] = 0.0;
  }
}

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// work space of nc vectors: a, bq [nc][npw] z64; sticks [nc][N][nst] z64;
// part [nsplit][nc][nproj] z64; C [nc][nproj] z64; zeros [nc] double; ids [nc] int
size_t bytes_for(const System& s, int nc) {
  const size_t mp = std::max(s.nproj, 1);
  return 2 * up256((size_t)nc * s.npw * sizeof(z64)) +
         up256((size_t)nc * s.N * s.nst * sizeof(z64)) +
         up256((size_t)s.nsplit * nc * mp * sizeof(z64)) + up256((size_t)nc * mp * sizeof(z64)) +
         up256((size_t)nc * sizeof(double)) + up256((size_t)nc * sizeof(int));
}

}  // namespace

size_t noalloc_capacity() { return kNoAllocBytes; }

// Device address of the work-space array on the current device (`device`).
void noalloc_init(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch.count(device)) return;
  void* p = nullptr;
  STH_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  g_scratch[device] = static_cast<unsigned char*>(p);
}

void Context::apply_h_noalloc(int id, int nvec, const double* in, double* out,
                              hipStream_t stream) {
  if (nvec < 0 || (nvec > 0 && (!in || !out))) {
    set_error("apply_h_noalloc: nvec >= 0 and non-null device in/out required");
    throw Error(STH_E_INVALID);
  }
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(device_);
    if (it == g_scratch.end()) {
      set_error("apply_h_noalloc: work space of device %d not initialised", device_);
      throw Error(STH_E_INTERNAL);
    }
    base = it->second;
  }
  System* sp = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = systems_.find(id);
    if (it == systems_.end()) {
      set_error("unknown system id %d", id);
      throw Error(STH_E_NOT_FOUND);
    }
    sp = it->second.get();
  }
  System& s = *sp;
  if (bytes_for(s, 1) > kNoAllocBytes) {
    set_error("apply_h_noalloc: one vector of this system needs %zu bytes of work space, more "
              "than the %zu of the static array", bytes_for(s, 1), kNoAllocBytes);
    throw Error(STH_E_INVALID);
  }
  if (nvec == 0) return;
  STH_HIP_CHECK(hipSetDevice(device_));
  int cap = 1;
  while (cap < nvec && bytes_for(s, cap + 1) <= kNoAllocBytes) ++cap;
  const size_t mp = std::max(s.nproj, 1);
  unsigned char* p = base;
  auto take = [&](size_t b) {
    unsigned char* q = p;
    p += up256(b);
    return q;
  };
  z64* a = reinterpret_cast<z64*>(take((size_t)cap * s.npw * sizeof(z64)));
  z64* bq = reinterpret_cast<z64*>(take((size_t)cap * s.npw * sizeof(z64)));
  HView w;
  w.cap = cap;
  w.sticks = reinterpret_cast<z64*>(take((size_t)cap * s.N * s.nst * sizeof(z64)));
  w.part = reinterpret_cast<z64*>(take((size_t)s.nsplit * cap * mp * sizeof(z64)));
  w.C = reinterpret_cast<z64*>(take((size_t)cap * mp * sizeof(z64)));
  w.zeros = reinterpret_cast<double*>(take((size_t)cap * sizeof(double)));
  w.ids = reinterpret_cast<int*>(take((size_t)cap * sizeof(int)));
  hipLaunchKernelGGL(k_fill_lists, dim3((cap + 255) / 256), dim3(256), 0, stream, w.ids, w.zeros,
                     cap);
  const z64* zin = reinterpret_cast<const z64*>(in);
  z64* zout = reinterpret_cast<z64*>(out);
  for (int c0 = 0; c0 < nvec; c0 += cap) {
    const int nc = std::min(cap, nvec - c0);
    launch_permute_in(zin + (size_t)c0 * s.npw, s.npw, a, s.npw, s.d_perm.as<int>(), s.npw, nc,
                      stream);
    h_block_on(s, w, a, bq, nc, stream);
    launch_permute_out(bq, s.npw, zout + (size_t)c0 * s.npw, s.npw, s.d_perm.as<int>(), s.npw,
                       nc, stream);
  }
  STH_HIP_CHECK(hipGetLastError());
}

}  // namespace sth
