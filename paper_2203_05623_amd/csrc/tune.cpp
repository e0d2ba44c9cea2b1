// Autotuner of a resident system: FFT radix plan (per precision) and the
// split-K chunk of the projector GEMM, timed on the system's own slot batch.
//
// Results are cached as JSON lines in the file named by STH_TUNE_CACHE (if
// set), one object per line:
//   {"key": "gfx950 N=72 npw=22575 nst=973 M=384 slots=2048", "plan64": 0,
//    "plan32": 1, "kchunk": 2048}
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

bool cache_lookup(const std::string& key, int* p64, int* p32, int* kc) {
  const char* path = std::getenv("STH_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (std::fgets(line, sizeof(line), f)) {
    if (!std::strstr(line, pat.c_str())) continue;
    const char* q = std::strstr(line, "\"plan64\":");
    const char* r = std::strstr(line, "\"plan32\":");
    const char* t = std::strstr(line, "\"kchunk\":");
    if (q && r && t && std::sscanf(q, "\"plan64\": %d", p64) == 1 &&
        std::sscanf(r, "\"plan32\": %d", p32) == 1 && std::sscanf(t, "\"kchunk\": %d", kc) == 1)
      found = true;   // the last matching line wins
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, int p64, int p32, int kc) {
  const char* path = std::getenv("STH_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"plan64\": %d, \"plan32\": %d, \"kchunk\": %d}\n",
               key.c_str(), p64, p32, kc);
  std::fclose(f);
}

}  // namespace

void Context::autotune(System& s) {
  const std::string key = tune_key(s);
  int p64 = 0, p32 = 0, kc = s.kchunk;
  if (cache_lookup(key, &p64, &p32, &kc) && p64 >= 0 && p64 < kRadixPlansHost && p32 >= 0 &&
      p32 < kRadixPlansHost && kc >= s.kchunk) {
    s.g.plan[0] = p64;
    s.g.plan[1] = p32;
    s.kchunk = kc;
    s.nsplit = (s.npw + kc - 1) / kc;
    s.tuned_from_cache = 1;
    return;
  }
  // timing batch: the slot pool itself (zeroed), up to 256 columns
  const int n = std::min(s.nslots, 256);
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
  int best[2] = {0, 0};
  for (int k = 0; k < 2; ++k) {
    double bt = 1e300;
    for (int p = 0; p < kRadixPlansHost; ++p) {
      s.g.plan[k] = p;
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
      s.tune_ms[2 * k + p] = ms;
      if (ms < bt) {
        bt = ms;
        best[k] = p;
      }
    }
    s.g.plan[k] = best[k];
  }
  // split-K chunk of C = W^H P (the partial buffer was sized for the smallest)
  const int cand[3] = {s.kchunk, 2 * s.kchunk, 4 * s.kchunk};
  double bt = 1e300;
  int bk = s.kchunk;
  for (int i = 0; i < 3; ++i) {
    const int kci = cand[i];
    const double ms = time_ms([&] {
      launch_gemm_ah_b(s.W(), s.npw, s.M, s.cvec(s.d_p), dl, n, s.npw, kci, s.d_part.as<z64>(),
                       st_);
      launch_reduce_parts(s.d_part.as<z64>(), (s.npw + kci - 1) / kci, n, s.M,
                          s.d_diag.as<double>(), 1.0, s.d_C.as<z64>(), st_);
    });
    s.tune_ms[4 + i] = ms;
    if (ms < bt) {
      bt = ms;
      bk = kci;
    }
  }
  s.kchunk = bk;
  s.nsplit = (s.npw + bk - 1) / bk;
  STH_HIP_CHECK(hipEventDestroy(a));
  STH_HIP_CHECK(hipEventDestroy(b));
  cache_store(key, s.g.plan[0], s.g.plan[1], s.kchunk);
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
  info->gemm_kchunk = s.kchunk;
  for (int i = 0; i < 8; ++i) info->tune_ms[i] = s.tune_ms[i];
  info->tuned_from_cache = s.tuned_from_cache;
}

}  // namespace sth
