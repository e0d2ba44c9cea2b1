// Autotuner of a resident system: FFT radix plan and plane kernel variant (per
// precision) and the split-K chunk of the projector GEMM, timed on the system's
// own slot batch.
//
// Results are cached as JSON lines in the file named by STH_TUNE_CACHE (if
// set), one object per line:
//   {"key": "gfx950 N=72 npw=22575 nst=973 M=384 slots=2048", "plan64": 1,
//    "kind64": 1, "zkind64": 0, "plan32": 1, "kind32": 0, "zkind32": 1, "kchunk": 1888}
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "engine.hpp"

namespace sth {

namespace {

std::string tune_key(const System& s) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "gfx950 N=%d npw=%d nst=%d M=%d slots=%d", s.N, s.npw, s.nst,
                s.M, s.nslots);
  return buf;
}

struct Choice {
  int plan[2] = {0, 0};
  int kind[2] = {0, 0};
  int zkind[2] = {0, 0};
  int kchunk = 0;
};

bool cache_lookup(const std::string& key, Choice* c) {
  const char* path = std::getenv("STH_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  auto field = [](const char* line, const char* name, int* out) {
    const std::string tag = std::string("\"") + name + "\": %d";
    const char* q = std::strstr(line, (std::string("\"") + name + "\":").c_str());
    return q && std::sscanf(q, tag.c_str(), out) == 1;
  };
  while (std::fgets(line, sizeof(line), f)) {
    if (!std::strstr(line, pat.c_str())) continue;
    Choice t;
    if (field(line, "plan64", &t.plan[0]) && field(line, "kind64", &t.kind[0]) &&
        field(line, "zkind64", &t.zkind[0]) && field(line, "plan32", &t.plan[1]) &&
        field(line, "kind32", &t.kind[1]) && field(line, "zkind32", &t.zkind[1]) &&
        field(line, "kchunk", &t.kchunk)) {
      *c = t;   // the last matching line wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const Choice& c) {
  const char* path = std::getenv("STH_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"plan64\": %d, \"kind64\": %d, \"zkind64\": %d, "
               "\"plan32\": %d, \"kind32\": %d, \"zkind32\": %d, \"kchunk\": %d}\n",
               key.c_str(), c.plan[0], c.kind[0], c.zkind[0], c.plan[1], c.kind[1], c.zkind[1],
               c.kchunk);
  std::fclose(f);
}

}  // namespace

void Context::autotune(System& s) {
  const std::string key = tune_key(s);
  Choice c;
  if (cache_lookup(key, &c)) {
    bool ok = c.kchunk >= s.kchunk;
    for (int k = 0; k < 2; ++k)
      ok = ok && c.plan[k] >= 0 && c.plan[k] < kRadixPlansHost && c.kind[k] >= 0 &&
           c.kind[k] < kPlaneKinds && c.zkind[k] >= 0 && c.zkind[k] < kZfftKinds &&
           plane_kind_available(s.g, c.kind[k], k == 1);
    if (ok) {
      for (int k = 0; k < 2; ++k) {
        s.g.plan[k] = c.plan[k];
        s.g.plane_kind[k] = c.kind[k];
        s.g.zfft_kind[k] = c.zkind[k];
      }
      s.kchunk = c.kchunk;
      s.nsplit = (s.npw + c.kchunk - 1) / c.kchunk;
      s.tuned_from_cache = 1;
      return;
    }
  }
  // timing batch: the whole slot pool (zeroed), the batch a CG step launches on
  const int n = s.nslots;
  s.d_p.zero(st_);
  s.d_q.zero(st_);
  s.d_sticks.zero(st_);
  const int* dl = s.d_ident.as<int>();
  hipEvent_t a, b;
  STH_HIP_CHECK(hipEventCreate(&a));
  STH_HIP_CHECK(hipEventCreate(&b));
  auto time_ms = [&](auto&& fn) {
    fn();   // warm-up
    STH_HIP_CHECK(hipEventRecord(a, st_));
    for (int r = 0; r < 3; ++r) fn();
    STH_HIP_CHECK(hipEventRecord(b, st_));
    STH_HIP_CHECK(hipEventSynchronize(b));
    float ms = 0.0f;
    STH_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    return double(ms) / 3.0;
  };
  const int N = s.N;
  VecSet<z64> st64{s.d_sticks.as<z64>(), (long long)N * s.nst};
  VecSet<z32> st32{reinterpret_cast<z32*>(s.d_sticks.as<z64>()), (long long)N * s.nst};
  // FFT stages of H psi for every (radix plan, plane kernel form, z-stick kernel
  // form), per precision; grids whose plane tile exceeds the LDS have the strip
  // form only

  for (int k = 0; k < 2; ++k) {
    double bt = 1e300;
    int bp = 0, bkind = kPlaneStrips, bz = 0;
    for (int zk = 0; zk < kZfftKinds; ++zk) {
      for (int kind = 0; kind < kPlaneKinds; ++kind) {
        if (!plane_kind_available(s.g, kind, k == 1)) continue;
        for (int p = 0; p < kRadixPlansHost; ++p) {
          s.g.plan[k] = p;
          s.g.plane_kind[k] = kind;
          s.g.zfft_kind[k] = zk;
          const double ms = time_ms([&] {
            if (k == 0) {
              launch_zfft_inv<double, z64>(s.g, s.cvec(s.d_p), st64, dl, n, st_);
              launch_plane_local<double>(s.g, st64, dl, n, s.d_vloc.as<double>(), nullptr, st_);
              launch_zfft_fwd<double, z64>(s.g, {st64.base, st64.stride}, s.vec(s.d_q), dl, n,
                                           ZF_PLAIN, {nullptr, 0}, nullptr, st_);
            } else {
              launch_zfft_inv<float, z64>(s.g, s.cvec(s.d_p), st32, dl, n, st_);
              launch_plane_local<float>(s.g, st32, dl, n, s.d_vloc32.as<float>(), nullptr, st_);
              launch_zfft_fwd<float, z64>(s.g, {st32.base, st32.stride}, s.vec(s.d_q), dl, n,
                                          ZF_PLAIN, {nullptr, 0}, nullptr, st_);
            }
          });
          s.tune_ms[20 * k + 10 * zk + 2 * kind + p] = ms;
          if (ms < bt) {
            bt = ms;
            bp = p;
            bkind = kind;
            bz = zk;
          }
        }
      }
    }
    s.g.plan[k] = bp;
    s.g.plane_kind[k] = bkind;
    s.g.zfft_kind[k] = bz;
  }
  // split-K chunk of C = W^H P (the partial buffer was sized for the smallest):
  // candidate split counts, so that the workgroup count can fill the 256 CUs evenly
  const int nsplits[8] = {kMaxSplit, 24, 16, 12, 11, 8, 6, 4};
  double bt = 1e300;
  int bk = s.kchunk, ncand = 0, prev = -1;
  for (int i = 0; i < 8; ++i) {
    const int kci = std::max(split_chunk(s.npw, nsplits[i]), s.kchunk);
    if (kci == prev) continue;
    prev = kci;
    const double ms = time_ms([&] {
      launch_gemm_ah_b(s.W(), s.npw, s.M, s.cvec(s.d_p), dl, n, s.npw, kci, s.d_part.as<z64>(),
                       st_);
      launch_reduce_parts(s.d_part.as<z64>(), (s.npw + kci - 1) / kci, n, s.M,
                          s.d_diag.as<double>(), 1.0, s.d_C.as<z64>(), st_);
    });
    s.tune_ms[40 + ncand++] = ms;
    if (ms < bt) {
      bt = ms;
      bk = kci;
    }
  }
  s.kchunk = bk;
  s.nsplit = (s.npw + bk - 1) / bk;
  STH_HIP_CHECK(hipEventDestroy(a));
  STH_HIP_CHECK(hipEventDestroy(b));
  for (int k = 0; k < 2; ++k) {
    c.plan[k] = s.g.plan[k];
    c.kind[k] = s.g.plane_kind[k];
    c.zkind[k] = s.g.zfft_kind[k];
  }
  c.kchunk = s.kchunk;
  cache_store(key, c);
}

void Context::system_info(int id, sth_system_info* info) {
  std::lock_guard<std::mutex> glk(gpu_mu_);
  System& s = sys(id);
  info->npw = s.npw;
  info->nsticks = s.nst;
  info->nslots = s.nslots;
  info->nv = s.nv;
  info->nproj = s.nproj;
  info->fft_plan_fp64 = s.g.plan[0];
  info->fft_plan_fp32 = s.g.plan[1];
  info->plane_kernel_fp64 = s.g.plane_kind[0];
  info->plane_kernel_fp32 = s.g.plane_kind[1];
  info->zfft_kernel_fp64 = s.g.zfft_kind[0];
  info->zfft_kernel_fp32 = s.g.zfft_kind[1];
  info->gemm_kchunk = s.kchunk;
  for (int i = 0; i < 48; ++i) info->tune_ms[i] = s.tune_ms[i];
  info->tuned_from_cache = s.tuned_from_cache;
  info->n = s.N;
  info->budget_used = budget_.used();
  info->budget_limit = budget_.limit();
}

}  // namespace sth
