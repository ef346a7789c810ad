// C ABI of the separable Helmholtz solver (declarations and contracts in
// include/helmsep.h).  Every entry point validates its arguments on the host,
// returns an hs_status and records a thread-local error text.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/helmsep.h"
#include "batch.hpp"
#include "plan.hpp"

struct hs_plan_s {
  hs::Plan p;
};

struct hs_batch_s {
  hs::Batch b;
};

namespace {
thread_local std::string g_err;

hs_status ret(hs_status s, const std::string& msg) {
  g_err = (s == HS_OK) ? std::string() : msg;
  return s;
}
}  // namespace

extern "C" {

const char* hs_status_str(hs_status s) {
  switch (s) {
    case HS_OK: return "HS_OK";
    case HS_ERR_ARG: return "HS_ERR_ARG";
    case HS_ERR_ALLOC: return "HS_ERR_ALLOC";
    case HS_ERR_DEVICE: return "HS_ERR_DEVICE";
    case HS_ERR_SINGULAR: return "HS_ERR_SINGULAR";
    case HS_ERR_NOCONV: return "HS_ERR_NOCONV";
    case HS_ERR_STATE: return "HS_ERR_STATE";
  }
  return "HS_ERR_UNKNOWN";
}

const char* hs_last_error(void) { return g_err.c_str(); }

hs_status hs_plan_create(const hs_grid* grid, const hs_blocks* blocks, const hs_options* opts, hs_plan* out) {
  if (!out) return ret(HS_ERR_ARG, "out is NULL");
  *out = nullptr;
  hs_plan p = new (std::nothrow) hs_plan_s;
  if (!p) return ret(HS_ERR_ALLOC, "host allocation failed");
  std::string err;
  hs_status s;
  try {
    s = p->p.build(grid, blocks, opts, err);
  } catch (const std::exception& e) {
    s = HS_ERR_ALLOC;
    err = e.what();
  }
  if (s != HS_OK) {
    delete p;
    return ret(s, err);
  }
  *out = p;
  return ret(HS_OK, "");
}

void hs_plan_destroy(hs_plan plan) { delete plan; }

size_t hs_plan_workspace_bytes(hs_plan plan, int32_t nrhs) {
  if (!plan || nrhs < 1 || nrhs > plan->p.max_rhs) return 0;
  return plan->p.ws_bytes;
}

hs_status hs_plan_bind_workspace(hs_plan plan, void* dev_ptr, size_t bytes) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.bind(dev_ptr, bytes, err), err);
}

hs_status hs_set_k2(hs_plan plan, const double* k2) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.set_k2(k2, err), err);
}

hs_status hs_solve(hs_plan plan, const void* f, void* u, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.solve(f, u, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_solve_adjoint(hs_plan plan, const void* g, void* a, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.solve_adjoint(g, a, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_grad_k2(hs_plan plan, const void* u, const void* a, void* grad, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.grad_k2(u, a, grad, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_grad_k2_noalloc(hs_plan plan, const void* u, const void* a, void* grad, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.grad_k2_noalloc(u, a, grad, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_residual(hs_plan plan, const void* f, const void* u, void* r, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.residual(f, u, r, 0, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_apply(hs_plan plan, const void* u, void* out, int32_t nrhs, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.residual(nullptr, u, out, 1, nrhs, (hipStream_t)stream, err), err);
}

hs_status hs_get_info(hs_plan plan, hs_info* info) {
  if (!plan || !info) return ret(HS_ERR_ARG, "plan or info is NULL");
  const hs::Plan& p = plan->p;
  std::memset(info, 0, sizeof(*info));
  info->nblocks = int32_t(p.blocks.size());
  info->refine_steps = p.refine_steps;
  for (auto& a : p.axes) {
    if (a.sine) ++info->n_sine_axes; else ++info->n_dense_axes;
    info->kappa_max = std::max(info->kappa_max, a.e.kappa);
    info->eig_resid_max = std::max(info->eig_resid_max, a.e.eig_resid);
    info->inv_resid_max = std::max(info->inv_resid_max, a.e.inv_resid);
  }
  info->min_pivot = p.min_pivot;
  info->plan_seconds = p.plan_seconds;
  info->table_bytes = p.tab_elems * (p.prec == 0 ? 16 : 24) + p.h16.size() * 2;
  info->n_fp64_modes = p.n_fp64_modes;
  info->z_chunks = hs::sweep_chunks_ok(p.tune_chunks, p.NZ) ? p.tune_chunks : hs::sweep_default_chunks(p.NZ);
  info->sine_lines = p.tune_lt;
  info->z_fixed_rows = p.tune_full;
  info->global_dense = p.dense_glob ? 1 : 0;
  info->fp64_stream = p.tune_side;
  for (auto& a : p.axes)
    if (a.hfwd >= 0) ++info->n_split_fp16;
  info->tol = p.tol;
  info->resid_first = -1;
  info->resid_final = -1;
  info->converged = -1;
  if (p.last_evals > 0) {
    std::vector<double> rel;
    int evals = 0, nrhs = 0;
    std::string err;
    hs_status s = p.residuals(rel, evals, nrhs, err);
    if (s != HS_OK) return ret(s, err);
    info->resid_evals = evals;
    double first = 0, last = 0;
    for (int r = 0; r < nrhs; ++r) {
      first = std::max(first, rel[r]);
      last = std::max(last, rel[size_t(evals - 1) * nrhs + r]);
    }
    info->resid_first = first;
    if (p.last_final) {
      info->resid_final = last;
      info->converged = last <= p.tol ? 1 : 0;
      if (!info->converged) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "last solve: relative residual %.3e above tol %.3e", last, p.tol);
        return ret(HS_ERR_NOCONV, buf);
      }
    }
  }
  return ret(HS_OK, "");
}

hs_status hs_get_residuals(hs_plan plan, double* rel, int32_t max_entries, int32_t* n_evals, int32_t* nrhs) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  if (max_entries < 0 || (max_entries > 0 && !rel)) return ret(HS_ERR_ARG, "rel is NULL");
  std::vector<double> v;
  int evals = 0, nr = 0;
  std::string err;
  hs_status s = plan->p.residuals(v, evals, nr, err);
  if (n_evals) *n_evals = evals;
  if (nrhs) *nrhs = nr;
  if (s != HS_OK) return ret(s, err);
  for (size_t i = 0; i < v.size() && i < size_t(max_entries); ++i) rel[i] = v[i];
  return ret(HS_OK, "");
}

hs_status hs_plan_tune(hs_plan plan, int32_t nrhs, const char* cache_path, void* stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.tune(nrhs, cache_path, (hipStream_t)stream, err), err);
}

hs_status hs_plan_set_coarse(hs_plan plan, hs_plan coarse) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  if (coarse == plan) return ret(HS_ERR_ARG, "a plan cannot be its own coarser plan");
  std::string err;
  return ret(plan->p.set_coarse(coarse ? &coarse->p : nullptr, err), err);
}

hs_status hs_plan_set_launch(hs_plan plan, int32_t z_chunks, int32_t sine_lines, int32_t z_fixed_rows,
                             int32_t global_dense, int32_t fp64_stream) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  hs::Plan& p = plan->p;
  if (z_chunks != 0 && !hs::sweep_chunks_ok(z_chunks, p.NZ)) return ret(HS_ERR_ARG, "z chunking cannot hold nz");
  if (sine_lines != 0) {
    for (auto& a : p.axes)
      if (a.dstV && !hs::dst_lt_ok(p.prec, a.dstV, sine_lines))
        return ret(HS_ERR_ARG, "sine lines per workgroup not usable on this plan");
    if (sine_lines != 4 && sine_lines != 8 && sine_lines != 16) return ret(HS_ERR_ARG, "sine lines not in {4, 8, 16}");
  }
  if (z_fixed_rows != 0 && z_fixed_rows != 1) return ret(HS_ERR_ARG, "z_fixed_rows not in {0, 1}");
  if (global_dense < -1 || global_dense > 1) return ret(HS_ERR_ARG, "global_dense not in {-1, 0, 1}");
  if (fp64_stream < -1 || fp64_stream > 1) return ret(HS_ERR_ARG, "fp64_stream not in {-1, 0, 1}");
  if (global_dense == 0 && p.decomposed && p.glob_forced)
    return ret(HS_ERR_ARG, "more than 4 separators on an axis (or flag bit 3): the global right-hand side is dense");
  if (global_dense >= 0) {
    std::string err;
    const hs_status st = p.set_global_dense(global_dense == 1, err);
    if (st != HS_OK) return ret(st, err);
  }
  p.tune_chunks = z_chunks;
  p.tune_lt = sine_lines;
  p.tune_full = z_fixed_rows;
  if (fp64_stream >= 0) p.tune_side = fp64_stream;
  return ret(HS_OK, "");
}

hs_status hs_profile_enable(hs_plan plan, int32_t on) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  return ret(plan->p.profile_enable(on != 0, err), err);
}

hs_status hs_profile_only(hs_plan plan, const char* stage) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  if (stage && std::strlen(stage) >= sizeof(hs_stage_time{}.name)) return ret(HS_ERR_ARG, "stage name too long");
  plan->p.prof_only = stage ? stage : "";
  return ret(HS_OK, "");
}

hs_status hs_profile_read(hs_plan plan, hs_stage_time* out, int32_t max_out, int32_t* n_out) {
  if (!plan) return ret(HS_ERR_ARG, "plan is NULL");
  std::string err;
  int n = 0;
  hs_status s = plan->p.profile_read(out, max_out, &n, err);
  if (n_out) *n_out = n;
  return ret(s, err);
}

hs_status hs_axis_eig(int32_t n, const double* h, double* lam, double* W, double* Winv, double* stats) {
  if (n < 1 || n > 4096 || !h || !lam || !W || !Winv) return ret(HS_ERR_ARG, "invalid arguments");
  std::vector<hs::cd> hv(n + 1);
  for (int i = 0; i <= n; ++i) {
    hv[i] = hs::cd(h[2 * i], h[2 * i + 1]);
    if (!(std::abs(hv[i]) > 0)) return ret(HS_ERR_ARG, "steps must be nonzero");
  }
  hs::AxisEig e;
  std::string err;
  if (hs::axis_is_uniform(n, hv.data())) {
    hs::axis_eig_uniform(n, hv[0], e);
  } else if (!hs::axis_eig_general(n, hv.data(), e, err)) {
    return ret(HS_ERR_SINGULAR, err);
  }
  std::memcpy(lam, e.lam.data(), sizeof(double) * 2 * n);
  std::memcpy(W, e.W.data(), sizeof(double) * 2 * size_t(n) * n);
  std::memcpy(Winv, e.Winv.data(), sizeof(double) * 2 * size_t(n) * n);
  if (stats) {
    stats[0] = e.kappa;
    stats[1] = e.eig_resid;
    stats[2] = e.inv_resid;
  }
  return ret(HS_OK, "");
}

// ---------------------------------------------------------------- batch

hs_status hs_batch_create(const hs_plan* plans, int32_t nplans, const int32_t* nrhs, hs_batch* out) {
  if (!out) return ret(HS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!plans || nplans < 1 || !nrhs) return ret(HS_ERR_ARG, "invalid plan list");
  std::vector<const hs::Plan*> ps(nplans);
  std::vector<int> rs(nplans);
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i]) return ret(HS_ERR_ARG, "NULL plan in list");
    ps[i] = &plans[i]->p;
    rs[i] = nrhs[i];
  }
  auto* b = new (std::nothrow) hs_batch_s;
  if (!b) return ret(HS_ERR_ALLOC, "host allocation failed");
  std::string err;
  hs_status s;
  try {
    s = b->b.build(ps, rs, err);
  } catch (const std::exception& e) {
    s = HS_ERR_ALLOC;
    err = e.what();
  }
  if (s != HS_OK) {
    delete b;
    return ret(s, err);
  }
  *out = b;
  return ret(HS_OK, "");
}

size_t hs_batch_workspace_bytes(hs_batch batch) { return batch ? batch->b.ws_bytes : 0; }

hs_status hs_batch_bind_workspace(hs_batch batch, void* dev_ptr, size_t bytes) {
  if (!batch) return ret(HS_ERR_ARG, "batch is NULL");
  std::string err;
  return ret(batch->b.bind(dev_ptr, bytes, err), err);
}

hs_status hs_batch_solve(hs_batch batch, const void* const* f, void* const* u, void* stream) {
  if (!batch) return ret(HS_ERR_ARG, "batch is NULL");
  std::string err;
  return ret(batch->b.solve(f, u, (hipStream_t)stream, err), err);
}

hs_status hs_batch_tune(hs_batch batch, const void* const* f, void* const* u, const char* cache_path, void* stream) {
  if (!batch) return ret(HS_ERR_ARG, "batch is NULL");
  if (!f || !u) return ret(HS_ERR_ARG, "f and u must be non-NULL");
  std::string err;
  return ret(batch->b.tune(f, u, cache_path, (hipStream_t)stream, err), err);
}

void hs_batch_destroy(hs_batch batch) { delete batch; }

}  // extern "C"
