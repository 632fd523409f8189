// C ABI of libpa (declared in include/pa.h): argument checks, error codes and
// the thread-local error message; no C++ exception crosses this boundary.
#include <atomic>
#include <cstring>
#include <string>

#include "pa_engine.h"

namespace pa {
std::string &last_error() {
  thread_local std::string msg;
  return msg;
}
uint64_t next_generation() {
  static std::atomic<uint64_t> counter{0};
  return ++counter;
}
}  // namespace pa

namespace {
using pa::guard;

void need(bool ok, const char *msg) {
  if (!ok) throw pa::Error(PA_EINVAL, msg);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// lp_min_cols that no column block reaches
constexpr int kLpNever = 1 << 30;
}  // namespace

extern "C" {

const char *pa_last_error(void) { return pa::last_error().c_str(); }

int pa_ctx_create(int device, void *stream, pa_ctx **out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    int n = 0;
    PA_HIP(hipGetDeviceCount(&n));
    need(device >= 0 && device < n, "device index out of range");
    auto *c = new pa_ctx;
    c->device = device;
    c->stream = (hipStream_t)stream;
    PA_HIP(hipSetDevice(device));
    hipError_t e = hipHostMalloc(&c->host_flag, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
      delete c;
      throw pa::Error(PA_EHIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *out = c;
  });
}

int pa_ctx_set_stream(pa_ctx *ctx, void *stream) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    ctx->stream = (hipStream_t)stream;
  });
}

int pa_ctx_profile(pa_ctx *ctx, int kernel) {
  return guard([&] {
    need(ctx != nullptr, "ctx is NULL");
    need(kernel >= PA_KERNEL_NONE && kernel <= PA_KERNEL_B2_STEP, "unknown kernel id");
    ctx->prof_kernel = kernel;
    ctx->prof_launches = ctx->prof_work = 0;
    ctx->prof_ms = ctx->prof_bytes = ctx->prof_units = 0.0;
  });
}

int pa_ctx_set_cg_budget(pa_ctx *ctx, double cg_rtol, int iters) {
  return guard([&] {
    need(ctx != nullptr && iters >= 0, "bad arguments");
    if (iters == 0)
      ctx->cg_budget.erase(cg_rtol);
    else
      ctx->cg_budget[cg_rtol] = iters;
  });
}

int pa_ctx_profile_read(pa_ctx *ctx, pa_kernel_profile *out) {
  return guard([&] {
    need(ctx && out, "NULL argument");
    out->launches = ctx->prof_launches;
    out->work_launches = ctx->prof_work;
    out->total_ms = ctx->prof_ms;
    out->bytes = ctx->prof_bytes;
    out->units = ctx->prof_units;
  });
}

int pa_ctx_destroy(pa_ctx *ctx) {
  return guard([&] {
    if (!ctx) return;
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->ev_a) (void)hipEventDestroy(ctx->ev_a);
    if (ctx->ev_b) (void)hipEventDestroy(ctx->ev_b);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
    if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
    delete ctx;
  });
}

int pa_mesh_icosahedral(int level, double radius, pa_mesh **out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    auto *m = new pa_mesh;
    try {
      m->m = pa::build_icosahedral(level, radius);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

int pa_mesh_get_info(const pa_mesh *m, pa_mesh_info *info) {
  return guard([&] {
    need(m && info, "NULL argument");
    info->level = m->m.level;
    info->nv = m->m.nv();
    info->ne = m->m.ne();
    info->nc = m->m.nc();
    info->radius = m->m.radius;
  });
}

int pa_mesh_export(const pa_mesh *m, double *verts, int32_t *cell_verts, int32_t *cell_edges,
                   int32_t *edge_cells, int32_t *edge_verts) {
  return guard([&] {
    need(m != nullptr, "mesh is NULL");
    const auto &M = m->m;
    if (verts) std::memcpy(verts, M.xyz.data(), M.xyz.size() * sizeof(double));
    if (cell_verts) std::memcpy(cell_verts, M.tri.data(), M.tri.size() * sizeof(int32_t));
    if (cell_edges) std::memcpy(cell_edges, M.cedge.data(), M.cedge.size() * sizeof(int32_t));
    if (edge_cells) std::memcpy(edge_cells, M.ecell.data(), M.ecell.size() * sizeof(int32_t));
    if (edge_verts) std::memcpy(edge_verts, M.evert.data(), M.evert.size() * sizeof(int32_t));
  });
}

int pa_mesh_destroy(pa_mesh *m) {
  return guard([&] { delete m; });
}

}  // extern "C"

namespace {
// Device layout of the operators: every array 256-byte aligned.
template <class T>
void place(size_t &off, const std::vector<T> &v, const T **dst, char *base) {
  off = align256(off);
  if (base) *dst = (const T *)(base + off);
  off += v.size() * sizeof(T);
}

size_t layout(pa_ops *o, char *base) {
  size_t off = 0;
  pa::DevOps d;
  place(off, o->ell_col, &d.ell_col, base);
  place(off, o->mass, &d.mass, base);
  place(off, o->cor, &d.cor, base);
  place(off, o->graddiv, &d.graddiv, base);
  place(off, o->mass32, &d.mass32, base);
  place(off, o->dinv, &d.dinv, base);
  place(off, o->dinv32, &d.dinv32, base);
  place(off, o->ecell, &d.ecell, base);
  place(off, o->cidx, &d.cidx, base);
  place(off, o->cell_edges, &d.cell_edges, base);
  place(off, o->tau, &d.tau, base);
  place(off, o->cedge, &d.cedge, base);
  place(off, o->csgn, &d.csgn, base);
  place(off, o->cnbr, &d.cnbr, base);
  place(off, o->area, &d.area, base);
  place(off, o->inv_area, &d.inv_area, base);
  place(off, o->bottom, &d.bottom, base);
  place(off, o->cgeo, &d.cgeo, base);
  place(off, o->nlform, &d.nlform, base);
  place(off, o->ring_cnt, &d.ring_cnt, base);
  place(off, o->ring_row, &d.ring_row, base);
  place(off, o->hloc, &d.hloc, base);
  place(off, o->ring_loc, &d.ring_loc, base);
  if (base) {
    d.hparts = o->hparts;
    d.fused_max = o->fused_max;
    d.ne = o->ne;
    d.nc = o->nc;
    d.g = o->g;
    d.H = o->H;
    o->d = d;
  }
  return align256(off);
}

template <class T>
void up(hipStream_t s, const T *dst, const std::vector<T> &v) {
  if (!v.empty())
    PA_HIP(hipMemcpyAsync((void *)dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}
}  // namespace

extern "C" {

int pa_ops_create(const pa_mesh *m, const pa_phys *ph, pa_ops **out) {
  return guard([&] {
    need(m && ph && out, "NULL argument");
    need(ph->g > 0 && ph->H > 0, "g and H must be positive");
    need(ph->lambda_bar >= 0, "lambda_bar must be >= 0");
    auto *o = new pa_ops;
    try {
      o->mesh = m;
      o->gen = pa::next_generation();
      pa::assemble_ops(o, m->m, *ph);
      o->dev_bytes = layout(o, nullptr);
    } catch (...) {
      delete o;
      throw;
    }
    *out = o;
  });
}

int pa_ops_device_size(const pa_ops *ops, size_t *bytes) {
  return guard([&] {
    need(ops && bytes, "NULL argument");
    *bytes = ops->dev_bytes;
  });
}

int pa_ops_bind(pa_ctx *ctx, pa_ops *ops, void *dev_buf) {
  return guard([&] {
    need(ctx && ops && dev_buf, "NULL argument");
    need(((uintptr_t)dev_buf & 255) == 0, "device buffer must be 256-byte aligned");
    PA_HIP(hipSetDevice(ctx->device));
    ops->dev = dev_buf;
    ops->gen = pa::next_generation();
    layout(ops, (char *)dev_buf);
    hipStream_t s = ctx->stream;
    const pa::DevOps &d = ops->d;
    up(s, d.ell_col, ops->ell_col);
    up(s, d.mass, ops->mass);
    up(s, d.cor, ops->cor);
    up(s, d.graddiv, ops->graddiv);
    up(s, d.mass32, ops->mass32);
    up(s, d.dinv, ops->dinv);
    up(s, d.dinv32, ops->dinv32);
    up(s, d.ecell, ops->ecell);
    up(s, d.cidx, ops->cidx);
    up(s, d.cell_edges, ops->cell_edges);
    up(s, d.tau, ops->tau);
    up(s, d.cedge, ops->cedge);
    up(s, d.csgn, ops->csgn);
    up(s, d.cnbr, ops->cnbr);
    up(s, d.area, ops->area);
    up(s, d.inv_area, ops->inv_area);
    up(s, d.bottom, ops->bottom);
    up(s, d.cgeo, ops->cgeo);
    up(s, d.nlform, ops->nlform);
    up(s, d.ring_cnt, ops->ring_cnt);
    up(s, d.ring_row, ops->ring_row);
    up(s, d.hloc, ops->hloc);
    up(s, d.ring_loc, ops->ring_loc);
    pa::sync_checked(s);
  });
}

int pa_ops_set_lambda(pa_ops *ops, double lambda_bar) {
  return guard([&] {
    need(ops != nullptr, "ops is NULL");
    need(lambda_bar > 0, "lambda_bar must be positive");
    ops->lambda_bar = lambda_bar;
  });
}

int pa_ops_get_lambda(const pa_ops *ops, double *lambda_bar) {
  return guard([&] {
    need(ops && lambda_bar, "NULL argument");
    *lambda_bar = ops->lambda_bar;
  });
}

int pa_ops_destroy(pa_ops *ops) {
  return guard([&] { delete ops; });
}

int pa_avg_create(int M, double T, pa_avg **out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    need(M >= 1 && T >= 0, "need M >= 1 and T >= 0");
    auto *a = new pa_avg;
    a->s.resize(M);
    a->w.resize(M);
    double sum = 0;
    for (int m = 0; m < M; m++) {
      const double x = -0.5 + (m + 0.5) / M;  // position in the support of rho
      a->s[m] = T * x;
      a->w[m] = std::exp(-1.0 / (0.25 - x * x));
      sum += a->w[m];
    }
    for (auto &w : a->w) w /= sum;
    *out = a;
  });
}

int pa_avg_create_nodes(int M, const double *s, const double *w, pa_avg **out) {
  return guard([&] {
    need(out && s && w && M >= 1, "bad arguments");
    auto *a = new pa_avg;
    a->s.assign(s, s + M);
    a->w.assign(w, w + M);
    *out = a;
  });
}

int pa_avg_nodes(const pa_avg *avg, double *s, double *w) {
  return guard([&] {
    need(avg != nullptr, "avg is NULL");
    if (s) std::memcpy(s, avg->s.data(), avg->s.size() * sizeof(double));
    if (w) std::memcpy(w, avg->w.data(), avg->w.size() * sizeof(double));
  });
}

int pa_avg_destroy(pa_avg *avg) {
  return guard([&] { delete avg; });
}

void pa_solve_cfg_default(pa_solve_cfg *cfg) {
  if (!cfg) return;
  cfg->precision = PA_FP64;
  cfg->backward = PA_BACKWARD_CLENSHAW;
  cfg->maxit = 100;
  cfg->growth_guard = 0;
  cfg->cg_rtol = 1e-10;
  cfg->cheb_tol = 1e-6;
  cfg->weight_cut = 1e-16;
  cfg->inner_rtol = 1e-6;
  cfg->use_graph = 1;
  cfg->solver = PA_SOLVER_CHEBYSHEV;
  cfg->precond = PA_PRECOND_JACOBI;
  cfg->exponential = PA_EXP_CHEBYSHEV;
  cfg->rexi_nodes = 0;
  cfg->rexi_eta0 = 0.0;
}

}  // extern "C"

namespace {
pa_solve_cfg cfg_or_default(const pa_solve_cfg *cfg) {
  pa_solve_cfg c;
  pa_solve_cfg_default(&c);
  return cfg ? *cfg : c;
}
}  // namespace

extern "C" {

}  // extern "C"

namespace pa {
// Workspace bytes of every call on `batch` states under configuration c
// (the planning code of the calls, run in its measuring mode).
size_t workspace_bytes(const pa_ops *ops, const pa_avg *avg, int batch, const pa_solve_cfg &c) {
  size_t best = 0;
  {
    // the rational exponential's node count follows the times of the call:
    // without a given node set, size for the largest (256 nodes)
    pa_solve_cfg ce = c;
    if (ce.exponential == PA_EXP_REXI && ce.rexi_nodes == 0) {
      ce.rexi_nodes = 256;
      ce.rexi_eta0 = 1.0;
    }
    pa::Engine e(nullptr, ops, ce, nullptr, 0);
    std::vector<double> t(batch, 1.0);
    if (ops->lambda_bar > 0) e.expL_apply(batch, t.data(), nullptr, nullptr);
    best = std::max(best, e.used());
  }
  {
    pa::Engine e(nullptr, ops, c, nullptr, 0);
    e.swe_nonlinear(batch, nullptr, nullptr);
    best = std::max(best, e.used());
  }
  {
    pa::Engine e(nullptr, ops, c, nullptr, 0);
    e.estimate_lambda(1);
    best = std::max(best, e.used());
  }
  {
    pa::Engine e(nullptr, ops, c, nullptr, 0);
    e.diagnostics(batch, nullptr, nullptr);
    best = std::max(best, e.used());
  }
  if (avg) {
    need(ops->lambda_bar > 0, "lambda_bar must be set before sizing averaged calls");
    pa::Engine e1(nullptr, ops, c, nullptr, 0);
    e1.phase_avg_rhs(avg, batch, nullptr, nullptr);
    best = std::max(best, e1.used());
    // the step's exponentials use the largest time step the caller may ask
    // for; size it by phase_avg_rhs plus stage buffers of a 2T step (with
    // the rational exponential the node count grows with the step: sized for
    // steps up to the averaging half-width max |s_m|)
    double T = 0;
    for (double s : avg->s) T = std::max(T, 2.0 * std::fabs(s));
    const double dt = c.exponential == PA_EXP_REXI ? 0.5 * T : T;
    pa::Engine e2(nullptr, ops, c, nullptr, 0);
    e2.step(avg, std::max(dt, 1.0), batch, nullptr);
    best = std::max(best, e2.used());
  }
  return best + 4096;
}
}  // namespace pa

extern "C" {

int pa_workspace_size(const pa_ops *ops, const pa_avg *avg, int batch, const pa_solve_cfg *cfg,
                      size_t *bytes) {
  return guard([&] {
    need(ops && bytes && batch >= 1, "bad arguments");
    *bytes = pa::workspace_bytes(ops, avg, batch, cfg_or_default(cfg));
  });
}

}  // extern "C"

namespace {
void check_call(pa_ctx *ctx, const pa_ops *ops, void *ws) {
  need(ctx && ops && ws, "NULL argument");
  need(ops->dev != nullptr, "operators not bound (pa_ops_bind)");
}
void out_stats(pa_stats *stats, const pa::Engine &e) {
  if (stats) *stats = e.stats;
}

// Repeats of the current call (budget overrun, failed Chebyshev check).
thread_local int g_repeats = 0;

// Run a call with the context's learned CG iteration budget when allowed
// (outputs not aliasing inputs); if a solve outlives the budget, run it
// again with host polling, which also relearns the budget.
template <class F>
void run_with_budget(pa_ctx *ctx, double rtol, bool allowed, F &&f) {
  if (allowed && ctx->cg_budget.count(rtol)) {
    try {
      f(true);
      return;
    } catch (const pa::BudgetExceeded &) {
      ctx->cg_budget.erase(rtol);
      g_repeats++;
    }
  }
  f(false);
}

// A Chebyshev mass solve whose final residual missed the tolerance makes
// the whole call run again with CG (possible only when outputs do not alias
// inputs; otherwise the failure is reported).
template <class F>
void run_with_fallback(pa_solve_cfg cfg, bool rerun_ok, F &&f) {
  try {
    f(cfg);
  } catch (const pa::SolverCheckFailed &) {
    if (!rerun_ok) throw;
    g_repeats++;
    cfg.solver = PA_SOLVER_CG;
    cfg.precision = PA_FP64;
    f(cfg);
  }
}
}  // namespace

namespace pa {
// The averaged right-hand side on a workspace, with the repeat rules (a
// budget overrun repeats with polling, a failed Chebyshev check with FP64
// CG when outputs do not alias inputs).
void phase_avg_rhs_call(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, int members,
                        const double *U_dev, double *Nbar_dev, void *ws, size_t ws_bytes,
                        const pa_solve_cfg &c0, pa_stats *stats) {
  need(avg && U_dev && Nbar_dev && members >= 1, "bad arguments");
  const bool may = U_dev != Nbar_dev;
  g_repeats = 0;
  run_with_fallback(c0, may, [&](const pa_solve_cfg &c) {
    run_with_budget(ctx, c.cg_rtol, may, [&](bool budget) {
      pa::Engine e(ctx, ops, c, ws, ws_bytes);
      e.allow_budget(budget, may);
      e.phase_avg_rhs(avg, members, U_dev, Nbar_dev);
      out_stats(stats, e);
    });
  });
  if (stats) stats->fallbacks = g_repeats;
}
}  // namespace pa

extern "C" {

int pa_ops_estimate_lambda(pa_ctx *ctx, pa_ops *ops, int iters, double safety, void *ws,
                           size_t ws_bytes, double *lambda_bar) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(iters >= 1 && safety >= 1.0, "need iters >= 1 and safety >= 1");
    pa_solve_cfg c;
    pa_solve_cfg_default(&c);
    c.cg_rtol = 1e-12;
    pa::Engine e(ctx, ops, c, ws, ws_bytes);
    const double rho = e.estimate_lambda(iters);
    ops->lambda_bar = safety * rho;
    if (lambda_bar) *lambda_bar = ops->lambda_bar;
  });
}

int pa_expL_apply(pa_ctx *ctx, const pa_ops *ops, int B, const double *t_host,
                  const double *U_in_dev, double *U_out_dev, void *ws, size_t ws_bytes,
                  const pa_solve_cfg *cfg, pa_stats *stats) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(t_host && U_in_dev && U_out_dev && B >= 1, "bad arguments");
    const pa_solve_cfg c0 = cfg_or_default(cfg);
    const bool may = U_in_dev != U_out_dev;
    g_repeats = 0;
    run_with_fallback(c0, may, [&](const pa_solve_cfg &c) {
      run_with_budget(ctx, c.cg_rtol, may, [&](bool budget) {
        pa::Engine e(ctx, ops, c, ws, ws_bytes);
        e.allow_budget(budget, may);
        e.expL_apply(B, t_host, U_in_dev, U_out_dev);
        out_stats(stats, e);
      });
    });
    if (stats) stats->fallbacks = g_repeats;
  });
}

int pa_swe_nonlinear(pa_ctx *ctx, const pa_ops *ops, int B, const double *U_dev, double *NU_dev,
                     void *ws, size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(U_dev && NU_dev && B >= 1, "bad arguments");
    const pa_solve_cfg c0 = cfg_or_default(cfg);
    const bool may = U_dev != NU_dev;
    g_repeats = 0;
    run_with_fallback(c0, may, [&](const pa_solve_cfg &c) {
      run_with_budget(ctx, c.cg_rtol, may, [&](bool budget) {
        pa::Engine e(ctx, ops, c, ws, ws_bytes);
        e.allow_budget(budget, may);
        e.swe_nonlinear(B, U_dev, NU_dev);
        out_stats(stats, e);
      });
    });
    if (stats) stats->fallbacks = g_repeats;
  });
}

int pa_phase_avg_rhs(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, int members,
                     const double *U_dev, double *Nbar_dev, void *ws, size_t ws_bytes,
                     const pa_solve_cfg *cfg, pa_stats *stats) {
  return guard([&] {
    check_call(ctx, ops, ws);
    pa::phase_avg_rhs_call(ctx, ops, avg, members, U_dev, Nbar_dev, ws, ws_bytes,
                           cfg_or_default(cfg), stats);
  });
}

int pa_step(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, double dt, int members,
            double *U_dev_inout, void *ws, size_t ws_bytes, const pa_solve_cfg *cfg,
            pa_stats *stats) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(avg && U_dev_inout && members >= 1 && dt > 0, "bad arguments");
    pa_solve_cfg c = cfg_or_default(cfg);
    c.solver = PA_SOLVER_CG;  // in place: no repeat possible, keep FP64 CG
    c.precision = PA_FP64;
    pa::Engine e(ctx, ops, c, ws, ws_bytes);
    e.step(avg, dt, members, U_dev_inout);
    out_stats(stats, e);
  });
}

}  // extern "C"

namespace {
void tune_out(const pa::LaunchTune &t, pa_launch_tune *out) {
  out->narrow_rows_per_thread = t.narrow_rows_per_thread;
  out->wide_max_wg = t.wide_max_wg;
  out->lp_min_cols = t.lp_min_cols;
  out->mixed_min_cols = t.mixed_min_cols;
  out->fused_steps = t.fused_steps;
  out->best_ms = 0.0;
}

pa::LaunchTune tune_in(const pa_launch_tune *t) {
  need(t->narrow_rows_per_thread >= 1 && t->narrow_rows_per_thread <= 64, "rows per thread in [1, 64]");
  need(t->wide_max_wg >= 8 && t->wide_max_wg <= 2048, "wide_max_wg in [8, 2048]");
  need(t->lp_min_cols >= 1 && t->mixed_min_cols >= 1, "lp_min_cols, mixed_min_cols >= 1");
  need(t->fused_steps >= 1 && t->fused_steps <= pa::kFusedMax, "fused_steps in [1, 6]");
  pa::LaunchTune lt;
  lt.narrow_rows_per_thread = t->narrow_rows_per_thread;
  lt.wide_max_wg = t->wide_max_wg;
  lt.lp_min_cols = t->lp_min_cols;
  lt.mixed_min_cols = t->mixed_min_cols;
  lt.fused_steps = t->fused_steps;
  return lt;
}
}  // namespace

extern "C" {

int pa_get_launch_tune(pa_launch_tune *out) {
  return guard([&] {
    need(out != nullptr, "out is NULL");
    tune_out(pa::launch_default(), out);
  });
}

int pa_set_launch_tune(const pa_launch_tune *t) {
  return guard([&] {
    need(t != nullptr, "t is NULL");
    pa::set_launch_default(tune_in(t));
  });
}

int pa_ops_set_tune(pa_ops *ops, const pa_launch_tune *t) {
  return guard([&] {
    need(ops != nullptr, "ops is NULL");
    if (t) {
      ops->tune = tune_in(t);
      ops->has_tune = true;
    } else {
      ops->has_tune = false;
    }
  });
}

int pa_ops_get_tune(const pa_ops *ops, pa_launch_tune *out, int *own) {
  return guard([&] {
    need(ops && out, "NULL argument");
    tune_out(ops->effective_tune(), out);
    if (own) *own = ops->has_tune ? 1 : 0;
  });
}

int pa_autotune(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, int members, const double *U_dev,
                double *out_dev, void *ws, size_t ws_bytes, const pa_solve_cfg *cfg,
                pa_launch_tune *out) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(avg && U_dev && out_dev && out && members >= 1 && U_dev != out_dev, "bad arguments");
    const pa_solve_cfg c = cfg_or_default(cfg);
    const pa::LaunchTune start = ops->effective_tune();
    const int rpts[] = {1, 2, 4, 8};
    const int caps[] = {512, 1024, 2048};
    double best = 1e300;
    pa::LaunchTune best_t = start;
    // one timed call in launch shape t (the operators' own shape is not
    // touched while searching)
    auto time_once = [&](const pa::LaunchTune &t) {
      pa_stats st{};
      run_with_fallback(c, true, [&](const pa_solve_cfg &cc) {
        run_with_budget(ctx, cc.cg_rtol, true, [&](bool budget) {
          pa::Engine e(ctx, ops, cc, ws, ws_bytes);
          e.set_tune(t);
          e.allow_budget(budget, true);
          e.phase_avg_rhs(avg, members, U_dev, out_dev);
          st = e.stats;
        });
      });
      return st.device_ms;
    };
    auto trial = [&](const pa::LaunchTune &t) {
      time_once(t);  // warm-up (and graph capture when enabled)
      double ms = std::min(time_once(t), time_once(t));
      if (ms < best) {
        best = ms;
        best_t = t;
      }
    };
    // the launch shape over rows per thread and workgroup caps, the other
    // fields as in `from`
    auto shapes = [&](const pa::LaunchTune &from) {
      for (int rpt : rpts)
        for (int cap : caps) {
          pa::LaunchTune t = from;
          t.narrow_rows_per_thread = rpt;
          t.wide_max_wg = cap;
          trial(t);
        }
    };
    shapes(start);
    auto search = [&](int pa::LaunchTune::*field, std::initializer_list<int> vals) {
      const pa::LaunchTune from = best_t;
      for (int v : vals) {
        pa::LaunchTune t = from;
        t.*field = v;
        trial(t);
      }
    };
    if (c.precond == PA_PRECOND_LEARNED) search(&pa::LaunchTune::lp_min_cols, {1, 8, 64, kLpNever});
    if (c.precision == PA_FP32_REFINED) search(&pa::LaunchTune::mixed_min_cols, {1, 8, 64, kLpNever});
    if (c.solver == PA_SOLVER_CHEBYSHEV) search(&pa::LaunchTune::fused_steps, {1, 2, 3, 4, 5, 6});
    // the shape again for the fields found (a learned threshold, a mixed
    // threshold or a step count can change which shape is fastest)
    shapes(best_t);
    ops->tune = best_t;
    ops->has_tune = true;
    tune_out(best_t, out);
    out->best_ms = best;
  });
}

int pa_diagnostics(pa_ctx *ctx, const pa_ops *ops, int B, const double *U_dev, void *ws,
                   size_t ws_bytes, double *out_host) {
  return guard([&] {
    check_call(ctx, ops, ws);
    need(U_dev && out_host && B >= 1, "bad arguments");
    pa_solve_cfg c;
    pa_solve_cfg_default(&c);
    pa::Engine e(ctx, ops, c, ws, ws_bytes);
    e.diagnostics(B, U_dev, out_host);
  });
}

}  // extern "C"
