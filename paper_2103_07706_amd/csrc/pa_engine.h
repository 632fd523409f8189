// Orchestration of libpa (internal): workspace planning and the enqueue-only
// sequences of kernels for the exponential, the nonlinearity, the averaged
// right-hand side and the RK4 step.
#pragma once
#include <complex>
#include <functional>
#include <vector>

#include "pa_kernels.h"
#include "pa_rexi.h"

namespace pa {

std::vector<double> bessel_weights(double theta, int kcap);
int truncate_degree(const std::vector<double> &c, double tol);
void assemble_ops(pa_ops *o, const Mesh &m, const pa_phys &ph);

// Workspace bytes of every call on `batch` states under configuration c.
size_t workspace_bytes(const pa_ops *ops, const pa_avg *avg, int batch, const pa_solve_cfg &c);
// pa_phase_avg_rhs on a given workspace (argument checks, repeat rules).
void phase_avg_rhs_call(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, int members,
                        const double *U_dev, double *Nbar_dev, void *ws, size_t ws_bytes,
                        const pa_solve_cfg &cfg, pa_stats *stats);

// Columns of a block: next power of two up to 64, then multiples of 64.
int pad_cols(int B);

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures (the same planning code sizes and carves the workspace).
// Raised when a solve still had active columns after the learned iteration
// budget; the call is then repeated with polling.
struct BudgetExceeded : Error {
  BudgetExceeded() : Error(PA_ENOCONV, "iteration budget exceeded") {}
};

// Raised when a Chebyshev mass solve missed its residual tolerance; the
// call is then repeated with CG.
struct SolverCheckFailed : Error {
  SolverCheckFailed() : Error(PA_ENOCONV, "Chebyshev mass solve missed the residual tolerance") {}
};

class Arena {
 public:
  Arena(void *base, size_t cap) : base_((char *)base), cap_(cap) {}
  template <class T>
  T *take(size_t n) {
    off_ = (off_ + 255) & ~(size_t)255;
    T *p = base_ ? (T *)(base_ + off_) : nullptr;
    off_ += n * sizeof(T);
    if (base_ && off_ > cap_) throw Error(PA_ENOMEM, "workspace too small");
    return p;
  }
  size_t used() const { return off_; }
  bool sizing() const { return base_ == nullptr; }

 private:
  char *base_;
  size_t cap_;
  size_t off_ = 0;
};

struct Blk {
  double *p = nullptr;
  int Bs = 0;
};

struct AccSpec {
  double *acc = nullptr;        // block with Bs / G columns
  const double *coef = nullptr; // Bs coefficients for this degree
  int acc_k = 0, G = 1;
};

// Chebyshev coefficient tables of one call.
struct ChebPlan {
  int kmax = 0;
  std::vector<int> K;  // per column
};

class Engine {
 public:
  Engine(pa_ctx *ctx, const pa_ops *ops, const pa_solve_cfg &cfg, void *ws, size_t ws_bytes);
  ~Engine();
  Engine(const Engine &) = delete;
  Engine &operator=(const Engine &) = delete;

  // planning + execution of the public calls (plan only when sizing)
  void expL_apply(int B, const double *t, const double *Uin, double *Uout);
  void swe_nonlinear(int B, const double *U, double *NU);
  void phase_avg_rhs(const pa_avg *avg, int members, const double *U, double *Nbar);
  void step(const pa_avg *avg, double dt, int members, double *U);
  double estimate_lambda(int iters);
  void diagnostics(int B, const double *U, double *out_host);

  size_t used() const { return ar_.used(); }

  // the same calls with every exponential the rational (REXI) sum
  // (cfg.exponential == PA_EXP_REXI; pa_rexi.cpp)
  void rexi_expL_apply(int B, const double *t, const double *Uin, double *Uout);
  void rexi_phase_avg_rhs(const pa_avg *avg, int members, const double *U, double *Nbar);
  void rexi_step(const pa_avg *avg, double dt, int members, double *U);

  // allow the learned CG iteration budget (no host polling) for this call
  // use: launch the learned budget without polling; learn: record the
  // largest iteration count of this call as the next budget
  void allow_budget(bool use, bool learn) {
    budget_ok_ = use;
    learn_budget_ = learn;
  }
  pa_stats stats{};

 private:
  struct NbarPlan;
  void plan_common(int BsMax);
  void begin();
  Blk block(int Bs);
  void lstep(Blk in, Blk out, const Blk *A, const Blk *B, double scale, const int *colK,
             int kneed, const AccSpec *acc);
  void cg(double *x, int Bs, const int *colK, int kneed, int nwg_init);
  void cheb_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init);
  void mass_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init);
  // residual checks of Chebyshev solves, deferred into the next set-up kernel
  double *chk_init_[2] = {nullptr, nullptr}, *chk_last_[2] = {nullptr, nullptr};
  int chk_par_ = 0;
  bool pend_ = false;
  CheckArgs pend_args_{};
  void defer_check(int Bs, int nwg_init, const int *colK, int kneed, int nwg_last = -1);
  // the set-up of a single-column solve done by its first fused launch
  struct FusedSetup {
    const double *in_u, *in_eta, *addA_u, *addA_eta, *addB_u, *addB_eta;
    double *out_eta;
    double scale;
  };
  void cheb_fused(double *x, const int *colK, int kneed, int nwg_init, int grid, int S,
                  const FusedSetup *su);
  unsigned long long fused_bytes(int n, int last, bool setup) const;
  int fused_setup_steps() const;  // steps per launch when lstep may fold its set-up, else 0
  void take_check(CheckArgs &chk, int &blocks, int grid_blocks);
  void flush_check();
  bool cheb() const { return cfg_.solver == PA_SOLVER_CHEBYSHEV; }
  bool mixed() const { return cfg_.precision == PA_FP32_REFINED; }
  void mixed_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init, bool prepared);
  std::vector<double> mix_c1_, mix_c2_;
  int mixed_outer_ = 0;
  int mixed_last_ = 0;  // steps of the last inner round (the others take mix_c1_.size())
  float *r32_ = nullptr, *d32_[2] = {nullptr, nullptr};
  // Chebyshev plan: step coefficients from the spectral bounds
  double cheb_theta_ = 0, cheb_delta_ = 0;
  // learned preconditioner plan (Chebyshev solves), chosen per solve
  bool lp_avail_ = false;
  double lp_theta_ = 0;
  std::vector<double> lp_c1_, lp_c2_;
  bool lp_cheaper(int Bs) const;
  bool lp_prof_wide_ = false;
  // growth guard: diagnostics of R_0 and R_kmax of up to kGuardSlots
  // averaged right-hand sides per call (the four of a step)
  static constexpr int kGuardSlots = 4;
  double *guard_ = nullptr;
  int guard_bm_ = 0, guard_members_ = 0, guard_calls_ = 0, guard_next_ = 0;  // measurement hook: form of the profiled learned steps
  std::vector<double> cheb_c1_, cheb_c2_;
  void plan_cheb();
  void poly_apply(Blk X, Blk W, const double *coef, const int *colK, int kmax, int G, Blk acc);
  void nonlinear_block(Blk E, Blk Y, const int *colK);
  void axpy(size_t n, double *out, double a0, const double *x0, double a1 = 0,
            const double *x1 = nullptr, double a2 = 0, const double *x2 = nullptr);
  void upload(void *dst, const void *src, size_t bytes);
  hipEvent_t take_event();
  void arm_events();
  void bracket_begin();
  void bracket_end(int n);
  struct ProfSpan {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int n = 0;  // launches between the two events
  };
  void diag(Blk X, double *out);
  std::vector<ProfSpan> prof_ev_;
  double prof_units_ = 0;  // fused mass-solve steps launched while profiling

  // phase average on a block of member columns X -> out (both [n][Bm])
 public:
  struct NbarBufs {
    int members = 0, Bm = 0, G = 0, BsE = 0, kmax = 0, M = 0;
    double *basis = nullptr, *E = nullptr, *Y = nullptr, *W = nullptr, *Z = nullptr;
    double *b1 = nullptr, *b2 = nullptr;
    double *cF = nullptr, *cB = nullptr, *cBx = nullptr;
    int *colK_E = nullptr, *colK_fwd = nullptr, *colK_mem = nullptr;
    std::vector<double> hcF, hcB, hcBx;
    std::vector<int> hcolK_E, hcolK_fwd, hcolK_mem;
    int ksum = 0;
  };
  struct NbarCall {
    NbarBufs nb;
    Blk X, out;
    const pa_avg *avg = nullptr;
    int members = 0;
    const double *U = nullptr;
    double *Nbar = nullptr;
  };
  // averaged RHS in pieces (used by batches of problems): plan the
  // workspace, enqueue the set-up on the caller's stream, enqueue the kernel
  // sequence on the engine's current stream, then finish()
  void nbar_plan(NbarCall &c, const pa_avg *avg, int members, const double *U, double *Nbar);
  void nbar_begin(NbarCall &c);
  void nbar_body(NbarCall &c);
  void finish();
  bool sync_free() const;
  int current_budget() const;
  void set_stream(hipStream_t s) { s_ = s; }
  // launch shape of this call's kernels (default: the operators' own shape,
  // else the process default)
  void set_tune(const LaunchTune &t) { tune_ = clamp_tune(t); }
  const LaunchTune &tune() const { return tune_; }
  hipStream_t stream() const { return s_; }

 private:
  void plan_nbar(NbarBufs &nb, const pa_avg *avg, int members);
  void upload_nbar(NbarBufs &nb);
  void run_nbar(NbarBufs &nb, Blk X, Blk out, bool uploaded);
  void run_graph(const GraphKey &key, const std::function<void()> &body);

  struct ExpBufs {
    int Bs = 0, kmax = 0;
    double *X = nullptr, *W = nullptr, *coef = nullptr;
    int *colK = nullptr;
    std::vector<double> hcoef;
    std::vector<int> hcolK;
  };
  void plan_exp(ExpBufs &eb, int B, const double *t);
  void run_exp(ExpBufs &eb, Blk in, Blk out);

  // rational exponential: one batch of shifted solves (P poles x members
  // complex columns) and its device buffers
  struct RexiSys {
    int N = 0, P = 0, members = 0, ncols = 0, Bc = 0, nwg = 0;
    double eta0 = 0.0;
    std::vector<std::complex<double>> X, W;  // poles, trapezoidal weights
    std::vector<double> hcoef;               // a, c, q, h, xinv per column
    double2 *coef = nullptr, *rho = nullptr, *alpha = nullptr, *omega = nullptr, *beta = nullptr;
    double *bb = nullptr, *ff = nullptr, *tau2 = nullptr, *res2 = nullptr, *part = nullptr;
    int *active = nullptr, *iters = nullptr, *fresh = nullptr, *restarts = nullptr, *fail = nullptr;
    double2 *Y = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr}, *v[2] = {nullptr, nullptr};
    double2 *s = nullptr, *t = nullptr;
    bool learned = false;  // left preconditioner P / X (else Jacobi)
    double2 *w = nullptr;  // learned form: the unpreconditioned vector
  };
  struct RexiExp {
    int B = 0, Bs = 0;
    std::vector<double2> hC;
    double2 *C = nullptr;
  };
  struct RexiNbar {
    int M = 0, G = 0, Bm = 0, BsE = 0, members = 0;
    std::vector<double2> hCf, hCb, hCs;
    std::vector<int> hcolK;
    double2 *Cf = nullptr, *Cb = nullptr, *Cs = nullptr, *Z = nullptr;
    int *colK = nullptr;
    double *E = nullptr, *Yn = nullptr;
  };
  void rexi_plan(RexiSys &rs, double theta_max, int members);
  void rexi_coefs(const RexiSys &rs, double theta, double scale, double2 *out) const;
  void rexi_upload(RexiSys &rs);
  void rexi_solve(RexiSys &rs, const RexiSrc &src);
  void rexi_combine(const RexiSys &rs, const double2 *C, int Go, int Mo, bool per_member, double *out,
                    int ostride);
  void rexi_exp_plan(RexiExp &x, RexiSys &rs, int B, const double *t);
  void rexi_exp_run(RexiExp &x, RexiSys &rs, Blk in, Blk out);
  double rexi_theta_max(const pa_avg *avg) const;
  void rexi_nbar_plan(RexiNbar &nb, RexiSys &rs, const pa_avg *avg, int members);
  void rexi_nbar_upload(RexiNbar &nb);
  void rexi_nbar_run(RexiNbar &nb, RexiSys &rs, Blk X, Blk out);

  pa_ctx *ctx_;
  const pa_ops *ops_;
  pa_solve_cfg cfg_;
  hipStream_t s_;
  int ne_, nc_, n_;
  Arena ar_;
  // CG scratch
  int BsMax_ = 0;
  double *r_ = nullptr, *r1_ = nullptr, *w0_ = nullptr, *w1_ = nullptr;
  double *s0_ = nullptr, *s1_ = nullptr, *p_ = nullptr;
  double *C_ = nullptr;
  SolveState st_{};
  RedBuf rb_{};
  unsigned *zero_base_ = nullptr;
  size_t zero_words_ = 0;
  int *colK0_ = nullptr;  // all zeros
  int predicted_ = 8;
  void *ws_base_ = nullptr;
  LaunchTune tune_;
  bool budget_ok_ = false, learn_budget_ = false;
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
};

}  // namespace pa
