// C ABI entry points (include/ipmg.h).  Every call catches internal errors and
// turns them into status codes with a per-context message.
#include <cmath>
#include <cstring>
#include <string>

#include "ctx.h"
#include "vec.h"

using ipmg::Ctx;
using ipmg::Error;

struct ipmg_ctx {
  Ctx c;
};

namespace {

template <class F>
int guard(ipmg_ctx* h, F&& fn) {
  if (!h) return IPMG_E_INVALID;
  try {
    const int rc = fn(h->c);
    if (rc == IPMG_OK) h->c.err.clear();
    return rc;
  } catch (const Error& e) {
    h->c.err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->c.err = "host allocation failed";
    return IPMG_E_NOMEM;
  } catch (const std::exception& e) {
    h->c.err = e.what();
    return IPMG_E_HIP;
  }
}

int check_level(const Ctx& c, int level) { return level >= 0 && level < c.L; }

}  // namespace

extern "C" {

int ipmg_create(const ipmg_desc* desc, void* hip_stream, ipmg_ctx** out) {
  if (!desc || !out) return IPMG_E_INVALID;
  *out = nullptr;
  ipmg_ctx* h = nullptr;
  try {
    h = new ipmg_ctx();
    ipmg::ctx_init(h->c, *desc, (hipStream_t)hip_stream);
  } catch (const Error& e) {
    if (h) { ipmg::ctx_free(h->c); delete h; }
    return e.code;
  } catch (...) {
    if (h) { ipmg::ctx_free(h->c); delete h; }
    return IPMG_E_NOMEM;
  }
  *out = h;
  return IPMG_OK;
}

void ipmg_destroy(ipmg_ctx* ctx) {
  if (!ctx) return;
  ipmg::ctx_free(ctx->c);
  delete ctx;
}

const char* ipmg_last_error(const ipmg_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

const char* ipmg_status_string(int s) {
  switch (s) {
    case IPMG_OK: return "ok";
    case IPMG_E_INVALID: return "invalid argument";
    case IPMG_E_DOMAIN: return "domain error";
    case IPMG_E_HIP: return "HIP runtime error";
    case IPMG_E_NOMEM: return "out of memory";
    case IPMG_E_BREAKDOWN: return "breakdown";
    case IPMG_E_NOT_CONVERGED: return "not converged";
    case IPMG_E_STALLED: return "interior-point step stalled";
    case IPMG_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int ipmg_sizes(const ipmg_ctx* ctx, int level, int64_t* n_slots, int64_t* n_free, int64_t* m_elems) {
  if (!ctx || !check_level(ctx->c, level)) return IPMG_E_INVALID;
  const ipmg::Dims& d = ctx->c.lev[level].d;
  if (n_slots) *n_slots = d.nslots;
  if (n_free) *n_free = d.nslots - (int64_t)ctx->c.dim * d.ny1 * d.nz1;
  if (m_elems) *m_elems = d.m;
  return IPMG_OK;
}

int ipmg_dof_map(const ipmg_ctx* ctx, int level, int64_t* free_to_slot) {
  if (!ctx || !free_to_slot || !check_level(ctx->c, level)) return IPMG_E_INVALID;
  const ipmg::Dims& d = ctx->c.lev[level].d;
  const int dim = ctx->c.dim;
  int64_t f = 0;
  for (int64_t s = 0; s < d.nslots; ++s) {
    const int64_t q = s / dim;
    if (q % d.nx1 != 0) free_to_slot[f++] = s;
  }
  return IPMG_OK;
}

int64_t ipmg_slot_of(const ipmg_ctx* ctx, int level, int i, int j, int k, int c) {
  if (!ctx || !check_level(ctx->c, level)) return -1;
  const ipmg::Dims& d = ctx->c.lev[level].d;
  const int dim = ctx->c.dim;
  if (i < 0 || i >= d.nx1 || j < 0 || j >= d.ny1 || k < 0 || k >= d.nz1 || c < 0 || c >= dim) return -1;
  return (((int64_t)k * d.ny1 + j) * d.nx1 + i) * dim + c;
}

int ipmg_element_matrix(ipmg_ctx* ctx, double* K0) {
  if (!K0) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    std::memcpy(K0, c.K0, sizeof(double) * c.nd * c.nd);
    return IPMG_OK;
  });
}

int ipmg_set_density(ipmg_ctx* ctx, const double* x) {
  if (!x) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::set_density(c, x);
    return IPMG_OK;
  });
}

int ipmg_apply_K(ipmg_ctx* ctx, const double* v, double* y) {
  if (!v || !y) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    if (!c.have_x) throw Error(IPMG_E_STATE, "set the densities first");
    const ipmg::Dims& d = c.fine();
    ipmg::vmask_copy(c.stream, v, c.pt, d.nslots, d.nslots, c.dim, d.nx1, c.red, ipmg::S_TMP0);
    c.ops->fine_apply64(c, IPMG_OP_K, c.pt, y, nullptr);
    IPMG_HIP(hipGetLastError());
    ipmg::sync(c);
    return IPMG_OK;
  });
}

int ipmg_apply_Z(ipmg_ctx* ctx, const double* v, double* y) {
  if (!v || !y) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    if (!c.have_z) throw Error(IPMG_E_STATE, "prepare the Newton system first");
    const ipmg::Dims& d = c.fine();
    ipmg::vmask_copy(c.stream, v, c.pt, d.nslots + 1, d.nslots, c.dim, d.nx1, c.red, ipmg::S_TMP0);
    c.ops->fine_apply64(c, IPMG_OP_Z, c.pt, y, nullptr);
    IPMG_HIP(hipGetLastError());
    ipmg::sync(c);
    return IPMG_OK;
  });
}

int ipmg_mg_setup(ipmg_ctx* ctx, int op) {
  if (op != IPMG_OP_K && op != IPMG_OP_Z) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::mg_setup(c, op, nullptr);
    return IPMG_OK;
  });
}

int ipmg_level_damping(ipmg_ctx* ctx, int level, double* omega, double* rho) {
  if (!omega || !rho) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    if (level < 0 || level >= c.L) throw Error(IPMG_E_INVALID, "bad level");
    IPMG_HIP(hipMemcpyAsync(omega, c.omega_dev + level, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    IPMG_HIP(hipMemcpyAsync(rho, c.omega_dev + c.L + level, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    ipmg::sync(c);
    if (level == 0) *rho = 0.0;
    return IPMG_OK;
  });
}

int ipmg_vcycle(ipmg_ctx* ctx, int op, const double* r, double* z) {
  if (!r || !z || (op != IPMG_OP_K && op != IPMG_OP_Z)) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::vcycle64(c, op, r, z);
    return IPMG_OK;
  });
}

int ipmg_pcg(ipmg_ctx* ctx, int op, const double* b, double* u, double rtol, int maxit, ipmg_pcg_info* info) {
  if (!b || !u || (op != IPMG_OP_K && op != IPMG_OP_Z)) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    if (op == IPMG_OP_Z && !c.have_z) throw Error(IPMG_E_STATE, "prepare the Newton system first");
    return ipmg::pcg(c, op, b, u, rtol, maxit, info);
  });
}

int ipmg_pcg_noalloc(ipmg_ctx* ctx, int op, const double* b, double* u, double rtol, int maxit,
                     ipmg_pcg_info* info) {
  if (!b || !u || (op != IPMG_OP_K && op != IPMG_OP_Z)) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    if (op == IPMG_OP_Z && !c.have_z) throw Error(IPMG_E_STATE, "prepare the Newton system first");
    return ipmg::pcg_noalloc(c, op, b, u, rtol, maxit, info);
  });
}

int64_t ipmg_pcg_noalloc_bytes(const ipmg_ctx* ctx) {
  if (!ctx) return -1;
  return (int64_t)ipmg::pcg_noalloc_bytes(ctx->c);
}

int ipmg_oc_update(ipmg_ctx* ctx, const double* u, const double* x, double V, double xbar, double q,
                   double lam_hi, double tau, const double* blend, double* x_new, ipmg_oc_info* info) {
  if (!u || !x || !x_new || x_new == x) return IPMG_E_INVALID;
  auto pos = [](double v) { return v > 0.0 && std::isfinite(v); };
  if (!pos(V) || !pos(xbar) || !pos(q) || !pos(lam_hi) || !pos(tau) || !(tau < lam_hi)) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::oc_update(c, u, x, V, xbar, q, lam_hi, tau, blend, x_new, info);
    return IPMG_OK;
  });
}

int ipmg_filter(ipmg_ctx* ctx, double rmin, const double* in, double* out, int transpose) {
  if (!in || !out || in == out || !(rmin > 0.0 && rmin <= 5.0) || (transpose != 0 && transpose != 1))
    return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    c.ops->filter(c, rmin, in, out, transpose);
    IPMG_HIP(hipGetLastError());
    ipmg::sync(c);
    return IPMG_OK;
  });
}

int ipmg_simp_compliance(ipmg_ctx* ctx, const double* x, const double* f, double rmin, double p, double rtol,
                         int maxit, double* u, double* grad, ipmg_pcg_info* info) {
  if (!x || !f || !u || !grad || !(rmin > 0.0 && rmin <= 5.0) || !(p >= 1.0 && std::isfinite(p)) ||
      !(rtol > 0.0) || maxit < 0)
    return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) { return ipmg::simp_compliance(c, x, f, rmin, p, rtol, maxit, u, grad, info); });
}

int ipmg_element_sens(ipmg_ctx* ctx, const double* w, const double* u, double scale, double* g) {
  if (!w || !u || !g) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    c.ops->element_sens(c, w, u, scale, g);
    IPMG_HIP(hipGetLastError());
    ipmg::sync(c);
    return IPMG_OK;
  });
}

int ipmg_profile_begin(ipmg_ctx* ctx, unsigned class_mask, int max_launches) {
  if (class_mask == 0 || class_mask >= (1u << ipmg::PC_COUNT) || max_launches < 1 || max_launches > (1 << 16))
    return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::sync(c);
    while ((int)c.prof_ev.size() < 2 * max_launches) {
      hipEvent_t e;   // timing only: no system-scope fence (no cache writeback around the kernel)
      IPMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      c.prof_ev.push_back(e);
    }
    c.prof_cls.assign(max_launches, -1);
    c.prof_mask = class_mask;
    c.prof_used = 0;
    return IPMG_OK;
  });
}

int ipmg_profile_end(ipmg_ctx* ctx, double* durations_ms, int* classes, int capacity, int* launches) {
  if (!launches || (capacity > 0 && !durations_ms)) return IPMG_E_INVALID;
  return guard(ctx, [&](Ctx& c) {
    ipmg::sync(c);
    const int n = c.prof_used;
    for (int i = 0; i < n && i < capacity; ++i) {
      float ms = 0.0f;
      IPMG_HIP(hipEventElapsedTime(&ms, c.prof_ev[2 * i], c.prof_ev[2 * i + 1]));
      durations_ms[i] = ms;
      if (classes) classes[i] = c.prof_cls[i];
    }
    *launches = n;
    c.prof_mask = 0;
    c.prof_used = 0;
    return IPMG_OK;
  });
}

static int check_ip(const ipmg_ip_params* p, const ipmg_ip_state* st) {
  if (!p || !st || !st->u || !st->x || !st->phi || !st->psi) return IPMG_E_INVALID;
  if (!(p->sigma > 0.0 && p->sigma < 1.0) || !(p->frac > 0.0 && p->frac < 1.0) || !(p->pcg_rtol > 0.0) ||
      p->pcg_maxit < 1 || !(p->xbar > 0.0) || !(p->accept_rtol >= 0.0))
    return IPMG_E_INVALID;
  return IPMG_OK;
}

int ipmg_ip_init(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, ipmg_ip_state* st,
                 ipmg_pcg_info* info) {
  if (!f) return IPMG_E_INVALID;
  const int v = check_ip(prm, st);
  if (v != IPMG_OK) return v;
  return guard(ctx, [&](Ctx& c) { return ipmg::ip_init(c, f, *prm, *st, info); });
}

int ipmg_ip_prepare(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, const ipmg_ip_state* st,
                    double* rhs) {
  if (!f) return IPMG_E_INVALID;
  const int v = check_ip(prm, st);
  if (v != IPMG_OK) return v;
  return guard(ctx, [&](Ctx& c) {
    ipmg::ip_prepare(c, f, *prm, *st);
    if (rhs) {
      IPMG_HIP(hipMemcpyAsync(rhs, c.ipRhs, sizeof(double) * (c.fine().nslots + 1), hipMemcpyDeviceToDevice,
                              c.stream));
      ipmg::sync(c);
    }
    return IPMG_OK;
  });
}

int ipmg_ip_step(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, ipmg_ip_state* st, ipmg_ip_info* info) {
  if (!f) return IPMG_E_INVALID;
  const int v = check_ip(prm, st);
  if (v != IPMG_OK) return v;
  return guard(ctx, [&](Ctx& c) { return ipmg::ip_step(c, f, *prm, *st, info); });
}

static bool simp_args_ok(double rmin, double pexp) {
  return rmin > 0.0 && rmin <= 5.0 && pexp >= 1.0 && std::isfinite(pexp);
}

int ipmg_simp_ip_init(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, double rmin, double pexp,
                      ipmg_ip_state* st, ipmg_pcg_info* info) {
  if (!f || !simp_args_ok(rmin, pexp)) return IPMG_E_INVALID;
  const int v = check_ip(prm, st);
  if (v != IPMG_OK) return v;
  return guard(ctx, [&](Ctx& c) { return ipmg::simp_ip_init(c, f, *prm, rmin, pexp, *st, info); });
}

int ipmg_simp_ip_step(ipmg_ctx* ctx, const double* f, const ipmg_ip_params* prm, double rmin, double pexp,
                      ipmg_ip_state* st, ipmg_ip_info* info) {
  if (!f || !simp_args_ok(rmin, pexp)) return IPMG_E_INVALID;
  const int v = check_ip(prm, st);
  if (v != IPMG_OK) return v;
  return guard(ctx, [&](Ctx& c) { return ipmg::simp_ip_step(c, f, *prm, rmin, pexp, *st, info); });
}

}  // extern "C"
