// C-ABI entry points: argument checks, error translation, thread-local message.
#include <cstdarg>
#include <cstdio>
#include <new>

#include "engine.hpp"

struct sth_ctx {
  sth::Context* impl;
};

namespace sth {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

}  // namespace sth

namespace {

template <typename F>
sth_status guard(F&& f) {
  try {
    sth::g_err[0] = '\0';
    f();
    return STH_OK;
  } catch (const sth::Error& e) {
    return static_cast<sth_status>(e.code);
  } catch (const std::bad_alloc&) {
    sth::set_error("host allocation failed");
    return STH_E_NOMEM;
  } catch (...) {
    sth::set_error("internal error");
    return STH_E_INTERNAL;
  }
}

sth::Context* ctx_of(sth_ctx* c) {
  if (!c || !c->impl) {
    sth::set_error("null context");
    throw sth::Error(STH_E_INVALID);
  }
  return c->impl;
}

void need(bool ok, const char* what) {
  if (!ok) {
    sth::set_error("invalid argument: %s", what);
    throw sth::Error(STH_E_INVALID);
  }
}

}  // namespace

extern "C" {

sth_status sth_create(const sth_config* cfg, sth_ctx** out) {
  return guard([&] {
    need(out != nullptr, "out");
    sth_config c{};
    if (cfg) c = *cfg;
    auto* h = new sth_ctx{nullptr};
    try {
      h->impl = new sth::Context(c);
    } catch (...) {
      delete h;
      throw;
    }
    *out = h;
  });
}

sth_status sth_destroy(sth_ctx* ctx) {
  return guard([&] {
    need(ctx != nullptr, "ctx");
    delete ctx->impl;
    delete ctx;
  });
}

sth_status sth_set_system(sth_ctx* ctx, const sth_system_desc* desc, void* stream,
                          int32_t* system_id) {
  return guard([&] {
    need(desc && system_id, "desc and system_id");
    *system_id = ctx_of(ctx)->set_system(*desc, static_cast<hipStream_t>(stream));
  });
}

sth_status sth_system_info_get(sth_ctx* ctx, int32_t system_id, sth_system_info* info) {
  return guard([&] {
    need(info != nullptr, "info");
    ctx_of(ctx)->system_info(system_id, info);
  });
}

sth_status sth_release_system(sth_ctx* ctx, int32_t system_id) {
  return guard([&] { ctx_of(ctx)->release_system(system_id); });
}

sth_status sth_apply_h(sth_ctx* ctx, int32_t system_id, int nvec, const double* in, double* out,
                       int ptr_kind, void* stream) {
  return guard([&] {
    ctx_of(ctx)->apply_h(system_id, nvec, in, out, ptr_kind, static_cast<hipStream_t>(stream));
  });
}

sth_status sth_apply_h_noalloc(sth_ctx* ctx, int32_t system_id, int nvec, const double* in,
                               double* out, void* stream) {
  return guard([&] {
    ctx_of(ctx)->apply_h_noalloc(system_id, nvec, in, out, static_cast<hipStream_t>(stream));
  });
}

sth_status sth_valence(sth_ctx* ctx, const sth_system_desc* desc, int nbands, double tol,
                       int maxit, double* eps_out, double* psi_out, int out_ptr_kind,
                       double* max_resid, int* iters) {
  return guard([&] {
    need(desc && eps_out && psi_out && nbands > 0 && tol > 0, "desc, outputs, nbands, tol");
    ctx_of(ctx)->valence(*desc, nbands, tol, maxit, eps_out, psi_out, out_ptr_kind, max_resid,
                         iters);
  });
}

sth_status sth_submit_solves(sth_ctx* ctx, int32_t system_id, int npert, const double* dv_r,
                             int nband, const int32_t* bands, const sth_solve_opts* opts,
                             int ptr_kind, void* stream, uint64_t* ticket) {
  return guard([&] {
    need(opts && ticket, "opts and ticket");
    *ticket = ctx_of(ctx)->submit(system_id, npert, dv_r, nband, bands, *opts, ptr_kind,
                                  static_cast<hipStream_t>(stream));
  });
}

sth_status sth_poll(sth_ctx* ctx, uint64_t ticket, sth_ticket_info* info) {
  return guard([&] {
    need(info != nullptr, "info");
    ctx_of(ctx)->poll(ticket, info);
  });
}

sth_status sth_wait(sth_ctx* ctx, uint64_t ticket, double timeout_s) {
  sth_status st = STH_OK;
  sth_status g = guard([&] {
    if (!ctx_of(ctx)->wait(ticket, timeout_s)) {
      sth::set_error("timeout waiting for ticket");
      st = STH_E_NOT_READY;
    }
  });
  return g != STH_OK ? g : st;
}

sth_status sth_fetch_drho(sth_ctx* ctx, uint64_t ticket, double* drho, int ptr_kind,
                          void* stream) {
  return guard([&] {
    need(drho != nullptr, "drho");
    ctx_of(ctx)->fetch_drho(ticket, drho, ptr_kind, static_cast<hipStream_t>(stream));
  });
}

sth_status sth_fetch_dpsi(sth_ctx* ctx, uint64_t ticket, double* dpsi, int ptr_kind,
                          void* stream) {
  return guard([&] {
    need(dpsi != nullptr, "dpsi");
    ctx_of(ctx)->fetch_dpsi(ticket, dpsi, ptr_kind, static_cast<hipStream_t>(stream));
  });
}

sth_status sth_fetch_stats(sth_ctx* ctx, uint64_t ticket, int32_t* iters, double* rel_resid,
                           int32_t* status, double* latency_s) {
  return guard([&] { ctx_of(ctx)->fetch_stats(ticket, iters, rel_resid, status, latency_s); });
}

sth_status sth_chi0_block(sth_ctx* ctx, uint64_t ticket, double* M, double* S, double* lambda) {
  return guard([&] { ctx_of(ctx)->chi0_block(ticket, M, S, lambda); });
}

sth_status sth_pdep(sth_ctx* ctx, int32_t system_id, int npdep, int nmax, double tol, int maxit,
                    double solve_tol, int precision, double* eig_out, double* vec_out,
                    int vec_ptr_kind, void* stream, int* iters, double* max_resid) {
  return guard([&] {
    need(eig_out != nullptr, "eig_out");
    ctx_of(ctx)->pdep(system_id, npdep, nmax, tol, maxit, solve_tol, precision, eig_out, vec_out,
                      vec_ptr_kind, static_cast<hipStream_t>(stream), iters, max_resid);
  });
}

sth_status sth_lanczos(sth_ctx* ctx, int32_t system_id, int band, int nphi, const double* phi,
                       int ptr_kind, int nsteps, double* alpha, double* beta, double* d,
                       double* U, double* braket, void* stream) {
  return guard([&] {
    ctx_of(ctx)->lanczos(system_id, band, nphi, phi, ptr_kind, nsteps, alpha, beta, d, U, braket,
                         static_cast<hipStream_t>(stream));
  });
}

sth_status sth_release_ticket(sth_ctx* ctx, uint64_t ticket) {
  return guard([&] { ctx_of(ctx)->release_ticket(ticket); });
}

sth_status sth_profile(sth_ctx* ctx, int enable) {
  return guard([&] { ctx_of(ctx)->profile(enable != 0); });
}

sth_status sth_profile_read(sth_ctx* ctx, double* ms, long long* launches, double* bytes,
                            double* flops) {
  return guard([&] { ctx_of(ctx)->profile_read(ms, launches, bytes, flops); });
}

const char* sth_last_error(void) { return sth::g_err; }

}  // extern "C"
