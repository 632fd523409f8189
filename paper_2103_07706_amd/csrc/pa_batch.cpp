// Batches of averaged right-hand-side problems (declared in include/pa.h):
// several meshes and ensembles evaluated together, concurrently on streams
// owned by the batch and, when requested, captured into one HIP graph.
#include <cstring>
#include <memory>
#include <string>

#include "pa_engine.h"

struct pa_batch {
  std::vector<const pa_ops *> ops;
  std::vector<int> members;
  const pa_avg *avg = nullptr;
  std::vector<pa::LaunchTune> tune;
  std::vector<bool> tuned;  // false: use the process-wide shape
  int device = -1;
  std::vector<hipStream_t> streams;  // one per item
  std::vector<hipEvent_t> join;      // one per item
  hipEvent_t fork = nullptr, done = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> key;
  std::vector<pa_stats> graph_stats;

  int n() const { return (int)ops.size(); }
  // an item's own shape, else its operators' shape, else the process default
  pa::LaunchTune item_tune(int i) const { return tuned[i] ? tune[i] : ops[i]->effective_tune(); }

  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    for (auto s : streams) (void)hipStreamDestroy(s);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
    streams.clear();
    join.clear();
    fork = done = nullptr;
    key.clear();
  }
  ~pa_batch() { release(); }

  // streams and events live on one device; a context on another device
  // recreates them
  void ensure(int dev) {
    if (device == dev && (int)streams.size() == n()) return;
    release();
    PA_HIP(hipSetDevice(dev));
    device = dev;
    for (int i = 0; i < n(); i++) {
      hipStream_t s = nullptr;
      PA_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      streams.push_back(s);
      hipEvent_t e = nullptr;
      PA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      join.push_back(e);
    }
    PA_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    PA_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  }
};

namespace {
void bneed(bool ok, const char *msg) {
  if (!ok) throw pa::Error(PA_EINVAL, msg);
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

pa_solve_cfg cfg_or_default(const pa_solve_cfg *cfg) {
  pa_solve_cfg c;
  pa_solve_cfg_default(&c);
  return cfg ? *cfg : c;
}

// Workspace of one item: the larger of its needs under cfg and under the
// FP64 CG configuration that a failed Chebyshev check falls back to.
size_t item_bytes(const pa_batch *b, int i, const pa_solve_cfg &c) {
  size_t best = 0;
  pa_solve_cfg cg = c;
  cg.solver = PA_SOLVER_CG;
  cg.precision = PA_FP64;
  const pa_solve_cfg *both[2] = {&c, &cg};
  for (const pa_solve_cfg *cc : both) {
    pa::Engine e(nullptr, b->ops[i], *cc, nullptr, 0);
    pa::Engine::NbarCall call;
    e.nbar_plan(call, b->avg, b->members[i], nullptr, nullptr);
    best = std::max(best, e.used());
  }
  return al256(best + 4096);
}

std::vector<size_t> item_offsets(const pa_batch *b, const pa_solve_cfg &c, size_t *total) {
  std::vector<size_t> off(b->n() + 1, 0);
  for (int i = 0; i < b->n(); i++) off[i + 1] = off[i] + item_bytes(b, i, c);
  *total = off[b->n()];
  return off;
}

template <class T>
void put(std::vector<unsigned char> &k, const T &v) {
  const unsigned char *p = (const unsigned char *)&v;
  k.insert(k.end(), p, p + sizeof(T));
}

// Everything a captured batch depends on: a change recaptures.
std::vector<unsigned char> batch_key(const pa_batch *b, const double *const *U,
                                     double *const *Nbar, void *ws, const pa_solve_cfg &c,
                                     int budget) {
  std::vector<unsigned char> k;
  put(k, b->avg->gen);
  put(k, ws);
  put(k, c.precision);
  put(k, c.backward);
  put(k, c.maxit);
  put(k, c.growth_guard);
  put(k, c.cg_rtol);
  put(k, c.cheb_tol);
  put(k, c.weight_cut);
  put(k, c.inner_rtol);
  put(k, c.use_graph);
  put(k, c.solver);
  put(k, c.precond);
  put(k, budget);
  for (int i = 0; i < b->n(); i++) {
    put(k, b->ops[i]->gen);
    put(k, b->ops[i]->lambda_bar);
    put(k, b->members[i]);
    put(k, U[i]);
    put(k, Nbar[i]);
    const pa::LaunchTune t = b->item_tune(i);
    put(k, t.narrow_rows_per_thread);
    put(k, t.wide_max_wg);
    put(k, t.lp_min_cols);
    put(k, t.mixed_min_cols);
    put(k, t.fused_steps);
  }
  return k;
}

// One evaluation of every item.  budget: use the context's learned CG
// budget (no polling); learn: record the batch's largest iteration count.
void run_once(pa_ctx *ctx, pa_batch *b, const double *const *U, double *const *Nbar, char *ws,
              const std::vector<size_t> &off, const pa_solve_cfg &c, bool budget, bool learn,
              pa_stats *stats) {
  const int n = b->n();
  std::vector<std::unique_ptr<pa::Engine>> E(n);
  std::vector<pa::Engine::NbarCall> call(n);
  bool sync_free = true;
  for (int i = 0; i < n; i++) {
    E[i].reset(new pa::Engine(ctx, b->ops[i], c, ws + off[i], off[i + 1] - off[i]));
    E[i]->set_tune(b->item_tune(i));
    E[i]->allow_budget(budget, false);
    E[i]->nbar_plan(call[i], b->avg, b->members[i], U[i], Nbar[i]);
    sync_free = sync_free && E[i]->sync_free();
  }
  hipStream_t cs = ctx->stream;
  int max_iters = 0;
  bool graph = false;
  if (!sync_free || ctx->prof_kernel != PA_KERNEL_NONE) {
    // polled CG solves (or per-launch timing): items in turn on the context stream
    for (int i = 0; i < n; i++) {
      E[i]->nbar_begin(call[i]);
      E[i]->nbar_body(call[i]);
      E[i]->finish();
      max_iters = std::max(max_iters, E[i]->stats.cg_iters_max);
    }
  } else {
    b->ensure(ctx->device);
    for (int i = 0; i < n; i++) E[i]->nbar_begin(call[i]);
    auto enqueue = [&] {
      for (int i = 0; i < n; i++) {
        E[i]->set_stream(b->streams[i]);
        E[i]->nbar_body(call[i]);
        E[i]->set_stream(cs);
      }
    };
    hipStream_t s0 = b->streams[0];
    PA_HIP(hipEventRecord(b->fork, cs));
    if (c.use_graph) {
      graph = true;
      PA_HIP(hipStreamWaitEvent(s0, b->fork, 0));
      const int bud = E[0]->current_budget();
      std::vector<unsigned char> key = batch_key(b, U, Nbar, ws, c, bud);
      if (!(b->exec && b->key == key)) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
        b->key.clear();
        hipGraph_t g = nullptr;
        PA_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
        try {
          // the other item streams join the capture through an event of s0
          PA_HIP(hipEventRecord(b->join[0], s0));
          for (int i = 1; i < n; i++) PA_HIP(hipStreamWaitEvent(b->streams[i], b->join[0], 0));
          enqueue();
          for (int i = 1; i < n; i++) {
            PA_HIP(hipEventRecord(b->join[i], b->streams[i]));
            PA_HIP(hipStreamWaitEvent(s0, b->join[i], 0));
          }
        } catch (...) {
          (void)hipStreamEndCapture(s0, &g);
          if (g) (void)hipGraphDestroy(g);
          for (auto &e : E) e->set_stream(cs);
          throw;
        }
        PA_HIP(hipStreamEndCapture(s0, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
          throw pa::Error(PA_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        b->exec = ex;
        b->key = key;
        b->graph_stats.resize(n);
        for (int i = 0; i < n; i++) b->graph_stats[i] = E[i]->stats;
        for (int i = 0; i < n; i++) E[i]->stats.graph_captured = 1;
      } else {
        for (int i = 0; i < n; i++) E[i]->stats = b->graph_stats[i];
      }
      PA_HIP(hipGraphLaunch(b->exec, s0));
      PA_HIP(hipEventRecord(b->done, s0));
      PA_HIP(hipStreamWaitEvent(cs, b->done, 0));
    } else {
      for (int i = 0; i < n; i++) PA_HIP(hipStreamWaitEvent(b->streams[i], b->fork, 0));
      enqueue();
      for (int i = 0; i < n; i++) {
        PA_HIP(hipEventRecord(b->join[i], b->streams[i]));
        PA_HIP(hipStreamWaitEvent(cs, b->join[i], 0));
      }
    }
    for (int i = 0; i < n; i++) {
      E[i]->finish();
      max_iters = std::max(max_iters, E[i]->stats.cg_iters_max);
    }
  }
  if (learn && c.solver == PA_SOLVER_CG && c.precision == PA_FP64)
    ctx->cg_budget[c.cg_rtol] = std::min(c.maxit, max_iters + 2);
  for (int i = 0; i < n; i++) {
    E[i]->stats.graph = graph ? 1 : 0;
    if (stats) stats[i] = E[i]->stats;
  }
}

// Same repeat rules as the single-problem calls: a budget overrun repeats
// with polling; a failed Chebyshev check repeats with FP64 CG.
void run_batch(pa_ctx *ctx, pa_batch *b, const double *const *U, double *const *Nbar, void *ws,
               size_t ws_bytes, const pa_solve_cfg &c0, pa_stats *stats) {
  if (c0.exponential != PA_EXP_CHEBYSHEV)
    throw pa::Error(PA_ENOTSUP, "batches run the Chebyshev exponential only");
  size_t total = 0;
  const std::vector<size_t> off = item_offsets(b, c0, &total);
  if (ws_bytes < total) throw pa::Error(PA_ENOMEM, "workspace too small for the batch");
  bool may = true;
  for (int i = 0; i < b->n(); i++) {
    bneed(U[i] && Nbar[i], "NULL state pointer");
    may = may && (const double *)Nbar[i] != U[i];
  }
  int repeats = 0;
  auto with_budget = [&](const pa_solve_cfg &c) {
    const bool cg64 = c.solver == PA_SOLVER_CG && c.precision == PA_FP64;
    if (may && cg64 && ctx->cg_budget.count(c.cg_rtol)) {
      try {
        run_once(ctx, b, U, Nbar, (char *)ws, off, c, true, false, stats);
        return;
      } catch (const pa::BudgetExceeded &) {
        ctx->cg_budget.erase(c.cg_rtol);
        repeats++;
      }
    }
    run_once(ctx, b, U, Nbar, (char *)ws, off, c, false, may, stats);
  };
  try {
    with_budget(c0);
  } catch (const pa::SolverCheckFailed &) {
    if (!may) throw;
    repeats++;
    pa_solve_cfg c = c0;
    c.solver = PA_SOLVER_CG;
    c.precision = PA_FP64;
    with_budget(c);
  }
  if (stats)
    for (int i = 0; i < b->n(); i++) stats[i].fallbacks = repeats;
}
}  // namespace

extern "C" {

int pa_batch_create(int n_items, const pa_ops *const *ops, const int *members, const pa_avg *avg,
                    pa_batch **out) {
  return pa::guard([&] {
    bneed(out && ops && members && avg && n_items >= 1, "bad arguments");
    auto b = std::unique_ptr<pa_batch>(new pa_batch);
    for (int i = 0; i < n_items; i++) {
      bneed(ops[i] != nullptr && members[i] >= 1, "each item needs operators and members >= 1");
      b->ops.push_back(ops[i]);
      b->members.push_back(members[i]);
    }
    b->avg = avg;
    b->tune.assign(n_items, pa::LaunchTune{});
    b->tuned.assign(n_items, false);
    *out = b.release();
  });
}

int pa_batch_workspace_size(const pa_batch *b, const pa_solve_cfg *cfg, size_t *bytes) {
  return pa::guard([&] {
    bneed(b && bytes, "NULL argument");
    for (auto o : b->ops) bneed(o->lambda_bar > 0, "lambda_bar must be set before sizing");
    size_t total = 0;
    item_offsets(b, cfg_or_default(cfg), &total);
    *bytes = total;
  });
}

int pa_batch_run(pa_ctx *ctx, pa_batch *b, const double *const *U_dev, double *const *Nbar_dev,
                 void *ws, size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats) {
  const int rc = pa::guard([&] {
    bneed(ctx && b && U_dev && Nbar_dev && ws, "NULL argument");
    for (auto o : b->ops) bneed(o->dev != nullptr, "operators not bound (pa_ops_bind)");
    run_batch(ctx, b, U_dev, Nbar_dev, ws, ws_bytes, cfg_or_default(cfg), stats);
  });
  return rc;
}

int pa_batch_set_tune(pa_batch *b, int item, const pa_launch_tune *t) {
  return pa::guard([&] {
    bneed(b && t && item >= 0 && item < b->n(), "bad arguments");
    bneed(t->narrow_rows_per_thread >= 1 && t->narrow_rows_per_thread <= 64, "rows per thread in [1, 64]");
    bneed(t->wide_max_wg >= 8 && t->wide_max_wg <= 2048, "wide_max_wg in [8, 2048]");
    bneed(t->lp_min_cols >= 1 && t->mixed_min_cols >= 1, "lp_min_cols, mixed_min_cols >= 1");
    bneed(t->fused_steps >= 1 && t->fused_steps <= pa::kFusedMax, "fused_steps in [1, 6]");
    b->tune[item].narrow_rows_per_thread = t->narrow_rows_per_thread;
    b->tune[item].wide_max_wg = t->wide_max_wg;
    b->tune[item].lp_min_cols = t->lp_min_cols;
    b->tune[item].mixed_min_cols = t->mixed_min_cols;
    b->tune[item].fused_steps = t->fused_steps;
    b->tuned[item] = true;
  });
}

int pa_batch_get_tune(const pa_batch *b, int item, pa_launch_tune *out) {
  return pa::guard([&] {
    bneed(b && out && item >= 0 && item < b->n(), "bad arguments");
    const pa::LaunchTune t = b->item_tune(item);
    out->narrow_rows_per_thread = t.narrow_rows_per_thread;
    out->wide_max_wg = t.wide_max_wg;
    out->lp_min_cols = t.lp_min_cols;
    out->mixed_min_cols = t.mixed_min_cols;
    out->fused_steps = t.fused_steps;
    out->best_ms = 0.0;
  });
}

int pa_batch_autotune(pa_ctx *ctx, pa_batch *b, const double *const *U_dev,
                      double *const *Nbar_dev, void *ws, size_t ws_bytes, const pa_solve_cfg *cfg,
                      pa_launch_tune *out) {
  return pa::guard([&] {
    bneed(ctx && b && U_dev && Nbar_dev && ws, "NULL argument");
    const pa_solve_cfg c = cfg_or_default(cfg);
    size_t total = 0;
    const std::vector<size_t> off = item_offsets(b, c, &total);
    if (ws_bytes < total) throw pa::Error(PA_ENOMEM, "workspace too small for the batch");
    for (int i = 0; i < b->n(); i++) {
      bneed(U_dev[i] && Nbar_dev[i] && (const double *)Nbar_dev[i] != U_dev[i],
            "outputs must not alias inputs");
      // a one-item batch over this item's slice of the workspace
      pa_batch one;
      one.ops = {b->ops[i]};
      one.members = {b->members[i]};
      one.avg = b->avg;
      one.tune.assign(1, pa::LaunchTune{});
      one.tuned.assign(1, true);
      const double *u1[1] = {U_dev[i]};
      double *o1[1] = {Nbar_dev[i]};
      char *w1 = (char *)ws + off[i];
      const size_t wb = off[i + 1] - off[i];
      double best = 1e300;
      pa::LaunchTune best_t = b->item_tune(i);
      auto trial = [&](const pa::LaunchTune &t) {
        one.tune[0] = t;
        pa_stats st{};
        run_batch(ctx, &one, u1, o1, w1, wb, c, &st);  // warm-up / capture
        double ms = 1e300;
        for (int r = 0; r < 2; r++) {
          run_batch(ctx, &one, u1, o1, w1, wb, c, &st);
          ms = std::min(ms, (double)st.device_ms);
        }
        if (ms < best) {
          best = ms;
          best_t = t;
        }
      };
      auto shapes = [&](const pa::LaunchTune &from) {
        for (int rpt : {1, 2, 4, 8})
          for (int cap : {512, 1024, 2048}) {
            pa::LaunchTune t = from;
            t.narrow_rows_per_thread = rpt;
            t.wide_max_wg = cap;
            trial(t);
          }
      };
      shapes(b->item_tune(i));
      for (int lmin : {1, 8, 64, 1 << 30}) {
        pa::LaunchTune t = best_t;
        if (c.precond == PA_PRECOND_LEARNED) {
          t.lp_min_cols = lmin;
          trial(t);
        }
      }
      for (int lmin : {1, 8, 64, 1 << 30}) {
        pa::LaunchTune t = best_t;
        if (c.precision == PA_FP32_REFINED) {
          t.mixed_min_cols = lmin;
          trial(t);
        }
      }
      if (c.solver == PA_SOLVER_CHEBYSHEV)
        for (int ps = 1; ps <= pa::kFusedMax; ps++) {
          pa::LaunchTune t = best_t;
          t.fused_steps = ps;
          trial(t);
        }
      // the shape again for the fields found
      shapes(best_t);
      b->tune[i] = best_t;
      b->tuned[i] = true;
      if (out) {
        out[i].narrow_rows_per_thread = best_t.narrow_rows_per_thread;
        out[i].wide_max_wg = best_t.wide_max_wg;
        out[i].lp_min_cols = best_t.lp_min_cols;
        out[i].mixed_min_cols = best_t.mixed_min_cols;
        out[i].fused_steps = best_t.fused_steps;
        out[i].best_ms = best;
      }
    }
  });
}

int pa_batch_destroy(pa_batch *b) {
  return pa::guard([&] { delete b; });
}

}  // extern "C"
