// Orchestration of libpa: the sequences of kernels for the Chebyshev
// exponential (Sec. 2.4), the nonlinearity (Sec. 2.5), the phase-averaged
// right-hand side (Sec. 2.2) and the averaged Lawson RK4 step (Sec. 2.3).
//
// Real form of the paper's recurrence.  With Lbar = lambda_bar |t| the
// modified polynomials satisfy P_k(L t) = T_k(x), x = -i sgn(t) L / lambda_bar,
// and exp(i Lbar x) = sum_k (2 - delta_k0) i^k J_k(Lbar) T_k(x).  Writing
// R_k = i^k T_k(-i L / lambda_bar) U (real):
//   R_0 = U,  R_1 = L U / lambda_bar,  R_{k+1} = (2 / lambda_bar) L R_k + R_{k-1},
//   exp(t L) U ~ sum_k c_k(t) R_k,  c_k(t) = (2 - delta_k0) J_k(lambda_bar |t|) sgn(t)^k.
// The R_k do not depend on t, so all forward shifts of one state share one
// basis and differ only in the coefficients.
#include "pa_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pa {

int pad_cols(int B) {
  if (B <= 0) return 0;
  if (B <= 64) {
    int p = 1;
    while (p < B) p <<= 1;
    return p;
  }
  return (B + 63) / 64 * 64;
}

static int tiles_of(int Bs) { return Bs <= 64 ? 1 : Bs / 64; }

Engine::Engine(pa_ctx *ctx, const pa_ops *ops, const pa_solve_cfg &cfg, void *ws, size_t ws_bytes)
    : ctx_(ctx), ops_(ops), cfg_(cfg), s_(ctx ? ctx->stream : nullptr), ne_(ops->ne),
      nc_(ops->nc), n_(ops->ne + ops->nc), ar_(ws, ws_bytes), ws_base_(ws),
      tune_(ops->effective_tune()) {
  if (cfg_.maxit <= 0) throw Error(PA_EINVAL, "maxit must be positive");
  if (!(cfg_.cg_rtol > 0)) throw Error(PA_EINVAL, "cg_rtol must be positive");
  if (!(cfg_.cheb_tol > 0)) throw Error(PA_EINVAL, "cheb_tol must be positive");
  if (cfg_.precision != PA_FP64 && cfg_.precision != PA_FP32_REFINED)
    throw Error(PA_EINVAL, "unknown precision");
  if (cfg_.solver != PA_SOLVER_CG && cfg_.solver != PA_SOLVER_CHEBYSHEV)
    throw Error(PA_EINVAL, "unknown solver");
  if (mixed() && !(cfg_.inner_rtol > 0 && cfg_.inner_rtol < 1)) throw Error(PA_EINVAL, "inner_rtol in (0, 1)");
  if (cfg_.exponential != PA_EXP_CHEBYSHEV && cfg_.exponential != PA_EXP_REXI)
    throw Error(PA_EINVAL, "unknown exponential");
  if (cheb() || mixed()) plan_cheb();
}

Engine::~Engine() {
  if (ev0_) (void)hipEventDestroy(ev0_);
  if (ev1_) (void)hipEventDestroy(ev1_);
}

// Chebyshev semi-iteration on D^-1 M over [a, b] = the Ritz bounds of 200
// Lanczos steps widened by 1% below and 0.5% above (on these mass matrices
// 200 steps put both ends within rounding of the extreme eigenvalues, 120
// within 1e-6); the number of steps makes the Chebyshev error factor
// 2/T_k(theta/delta) reach cg_rtol, plus one.  Measured worst final
// residual at cg_rtol = 1e-10: about 1e-11.  The final FP64 residual check
// guards every solve.
namespace {
constexpr double kBoundLow = 0.99, kBoundHigh = 1.005;
int cheb_steps(double a, double b, double rtol) {
  const double sigma = (a + b) / (b - a);
  return (int)std::ceil(std::acosh(2.0 / rtol) / std::acosh(sigma)) + 1;
}
}  // namespace

namespace {
// Chebyshev semi-iteration coefficients over [a, b]: x += d_k, r -= M d_k,
// d_{k+1} = c1_k d_k + c2_k B r (B the preconditioner).
void cheb_coefs(double a, double b, int k, std::vector<double> &c1, std::vector<double> &c2) {
  const double theta = 0.5 * (a + b), delta = 0.5 * (b - a), sigma = theta / delta;
  c1.resize(k);
  c2.resize(k);
  double rho = 1.0 / sigma;
  for (int i = 0; i < k; i++) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[i] = rn * rho;
    c2[i] = 2.0 * rn / delta;
    rho = rn;
  }
}
}  // namespace

void Engine::plan_cheb() {
  const double a = kBoundLow * ops_->mass_eig_min, b = kBoundHigh * ops_->mass_eig_max;
  if (!(a > 0) || !(b > a)) throw Error(PA_EINVAL, "no spectral bounds for the mass matrix");
  if (cfg_.precond != PA_PRECOND_JACOBI && cfg_.precond != PA_PRECOND_LEARNED)
    throw Error(PA_EINVAL, "unknown preconditioner");
  // learned preconditioner: its own widened bounds; whether a solve uses it
  // is decided per solve by lp_cheaper()
  lp_avail_ = false;
  if (cfg_.precond == PA_PRECOND_LEARNED && cheb() && !mixed()) {
    if (!ops_->lp_ready || !ops_->lp_dev)
      throw Error(PA_EINVAL, "no learned preconditioner bound to the operators");
    const double la = kBoundLow * ops_->lp_eig_min, lb = kBoundHigh * ops_->lp_eig_max;
    if (la > 0 && lb > la) {
      lp_avail_ = true;
      lp_theta_ = 0.5 * (la + lb);
      cheb_coefs(la, lb, std::min(cheb_steps(la, lb, cfg_.cg_rtol), cfg_.maxit), lp_c1_, lp_c2_);
    }
  }
  cheb_theta_ = 0.5 * (a + b);
  cheb_delta_ = 0.5 * (b - a);
  const double sigma = cheb_theta_ / cheb_delta_;
  cheb_coefs(a, b, std::min(cheb_steps(a, b, cfg_.cg_rtol), cfg_.maxit), cheb_c1_, cheb_c2_);
  if (mixed()) {
    // FP32 inner solves to eps = max(inner_rtol, 1e-6) (single-precision
    // floor), outer FP64 refinements until eps^n_out reaches cg_rtol
    const double eps = std::max(cfg_.inner_rtol, 1e-6);
    const int kin = std::min(cfg_.maxit, (int)std::ceil(std::acosh(2.0 / eps) / std::acosh(sigma)) + 1);
    mixed_outer_ = std::max(1, (int)std::ceil(std::log(cfg_.cg_rtol) / std::log(10.0 * eps)));
    // the first kin coefficients of the same recurrence
    cheb_coefs(a, b, kin, mix_c1_, mix_c2_);
    // The round count assumes only 10 eps per round; a round of kin steps
    // reaches eps (its Chebyshev bound, above the FP32 floor), so the last
    // round needs only the rest, cg_rtol / eps^(rounds - 1), and takes the
    // steps of that bound (at least half a round).  The FP64 residual check
    // of every solve still decides.
    const double rest = cfg_.cg_rtol / std::pow(eps, mixed_outer_ - 1);
    int klast = kin;
    if (rest > eps && rest < 1.0)
      klast = (int)std::ceil(std::acosh(2.0 / rest) / std::acosh(sigma)) + 1;
    else if (rest >= 1.0)
      klast = 1;
    mixed_last_ = std::min(kin, std::max(klast, (kin + 1) / 2));
  }
}

// Mixed-precision mass solve (FP32 inner Chebyshev, FP64 refinement); the
// set-up kernel wrote r_0, x_0 and the partials of |r_0|^2 (partA).
void Engine::mixed_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init, bool prepared) {
  RefineArgs ra{};
  ra.ops = ops_->d;
  ra.Bs = Bs;
  ra.x = x;
  ra.r = r_;
  ra.x32 = nullptr;  // not read by the first refinement (first = 1)
  ra.r32 = r32_;
  ra.d32 = d32_[0];
  ra.theta_inv = (float)(1.0 / cheb_theta_);
  ra.colK = colK;
  ra.kneed = kneed;
  ra.part = chk_last_[chk_par_];
  ra.max_wg = rb_.max_wg;
  ra.first = 1;
  if (!prepared) launch_refine(ra, s_);
  // inner solves in the three-term form: the refinement writes b = r32 and
  // x_1 = D^-1 b / theta into the buffer `cur`; steps 1..kin-1 form
  // x_{i+1} over x_{i-1}; the next refinement reads x_kin and writes the next
  // round's x_1 into the other buffer
  Cheb32Args ca{};
  ca.ops = ops_->d;
  ca.Bs = Bs;
  ca.b32 = r32_;
  ca.colK = colK;
  ca.kneed = kneed;
  const int kin = (int)mix_c1_.size();
  float *cur = d32_[0], *prev = d32_[1];
  const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB32_ITER;
  ca.prof = prof ? st_.prof : nullptr;
  ca.prof_bytes = st_.prof_bytes;
  int steps = 0;
  for (int o = 0; o < mixed_outer_; o++) {
    const int kr = o + 1 == mixed_outer_ ? mixed_last_ : kin;
    steps += kr;
    if (prof && kr > 1) bracket_begin();
    for (int i = 1; i < kr; i++) {
      ca.x_cur = cur;
      ca.x_prev = prev;
      ca.x_next = prev;
      ca.c1 = (float)mix_c1_[i - 1];
      ca.c2 = (float)mix_c2_[i - 1];
      ca.zero_prev = i == 1 ? 1 : 0;
      launch_cheb32_iter(ca, s_);
      std::swap(cur, prev);
    }
    if (prof && kr > 1) bracket_end(kr - 1);
    ra.first = 0;
    ra.last = o + 1 == mixed_outer_ ? 1 : 0;
    ra.x_zero = prepared && o == 0 ? 1 : 0;  // the gather kernel left x unwritten
    ra.x32 = cur;
    ra.d32 = prev;  // the next x_1, beside the x_kin this kernel gathers
    launch_refine(ra, s_);
    std::swap(cur, prev);
  }
  defer_check(Bs, nwg_init, colK, kneed);
  stats.solves++;
  stats.refinements += mixed_outer_;
  stats.cg_iters += steps;
  stats.cg_iters_max = std::max(stats.cg_iters_max, steps);
}

// Reduction-free mass solve: the set-up kernel wrote r_0 (r), x_0 (x),
// d_0 = D^-1 r_0 / theta (p) and partials of |r_0|^2 (partA).
// Residual check of the solve just enqueued: deferred to the next set-up
// kernel (take_check) or to flush_check at the end of the call.
void Engine::defer_check(int Bs, int nwg_init, const int *colK, int kneed, int nwg_last) {
  CheckArgs &ck = pend_args_;
  ck = CheckArgs{};
  ck.Bs = Bs;
  ck.nwg_init = nwg_init;
  ck.nwg_last = nwg_last >= 0 ? nwg_last : launch_rows_grid(ne_, Bs);
  ck.max_wg = rb_.max_wg;
  ck.part_init = chk_init_[chk_par_];
  ck.part_last = chk_last_[chk_par_];
  ck.colK = colK;
  ck.kneed = kneed;
  ck.rtol2 = cfg_.cg_rtol * cfg_.cg_rtol;
  ck.fail = st_.cheb_fail;
  ck.resid = st_.resid;
  ck.resid_max = st_.resid_max;
  pend_ = true;
  chk_par_ ^= 1;
}

// Hands the pending check to a set-up kernel of `grid_blocks` workgroups
// (enough for the check), else launches it on its own first.
void Engine::take_check(CheckArgs &chk, int &blocks, int grid_blocks) {
  blocks = 0;
  if (!pend_) return;
  const int need = cheb_check_blocks(pend_args_);
  if (grid_blocks >= need) {
    chk = pend_args_;
    blocks = need;
    pend_ = false;
  } else {
    flush_check();
  }
}

void Engine::flush_check() {
  if (!pend_) return;
  launch_cheb_check(pend_args_, s_);
  pend_ = false;
}

// The mass solve after a set-up kernel.  With FP32 refinement enabled, the
// refined solve runs on blocks at least mixed_min_cols wide (its FP32 steps
// halve the bytes of a step, which pays where steps are bandwidth bound);
// narrower blocks, whose steps are launch-latency bound, take FP64 steps.
void Engine::mass_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init) {
  if (mixed() && Bs >= tune_.mixed_min_cols)
    mixed_solve(x, Bs, colK, kneed, nwg_init, false);
  else if (cheb() || mixed())
    cheb_solve(x, Bs, colK, kneed, nwg_init);
  else
    cg(x, Bs, colK, kneed, nwg_init);
}

// Learned or Jacobi steps for a solve on Bs columns.  A learned step moves
// more bytes than a Jacobi step (the P and P M rows, and gathers over two and
// three rings of neighbours against one), so fewer steps pay only on wide
// enough blocks; the threshold is part of the launch shape, which the
// autotuner measures.
bool Engine::lp_cheaper(int Bs) const { return lp_avail_ && Bs >= tune_.lp_min_cols; }

// Jacobi semi-iteration of a single column, S steps per launch
// (k_cheb_fused): the remainder of the step count first, then launches of S
// steps.  r and d move between two buffers each from one launch to the next.
// With `su`, the first launch also does the set-up of the solve (the work of
// k_stiff) as its step 1 and then as many Chebyshev steps as the remainder
// (at most S - 1).
void Engine::cheb_fused(double *x, const int *colK, int kneed, int nwg_init, int grid, int S,
                        const FusedSetup *su) {
  const std::vector<double> &c1 = cheb_c1_, &c2 = cheb_c2_;
  const int k = (int)c1.size();
  double *d[2] = {p_, s0_};
  double *r[2] = {r_, r1_};
  ChebFusedArgs a{};
  a.ops = ops_->d;
  a.x = x;
  a.colK = colK;
  a.kneed = kneed;
  a.part = chk_last_[chk_par_];
  const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB_FUSED;
  a.prof = prof ? st_.prof : nullptr;
  a.prof_bytes = st_.prof_bytes;
  int launches = 0, i = 0, buf = 0, setup_grid = grid;
  if (prof) bracket_begin();
  if (su) {
    int c = k % S ? k % S : S - 1;
    c = std::min(c, k);
    ChebFusedArgs b = a;
    b.setup = 1;
    b.S = c + 1;
    for (int st = 0; st < kFusedMax; st++) b.slots[st] = ops_->fused_slots[c + 1][st];
    for (int st = 1; st <= c; st++) {
      b.c1[st] = c1[st - 1];
      b.c2[st] = c2[st - 1];
    }
    b.in_u = su->in_u;
    b.in_eta = su->in_eta;
    b.addA_u = su->addA_u;
    b.addA_eta = su->addA_eta;
    b.addB_u = su->addB_u;
    b.addB_eta = su->addB_eta;
    b.out_eta = su->out_eta;
    b.scale = su->scale;
    b.theta_inv = 1.0 / cheb_theta_;
    b.cpp = ops_->fused_cpp;
    b.part_rr = chk_init_[chk_par_];
    // the pending check gets workgroups of its own past the parts when the
    // grid has room for them
    take_check(b.chk, b.chk_blocks, launch_max_wg() - grid);
    setup_grid = cheb_fused_grid(ops_->d, b.chk_blocks);
    b.r_out = r[1];
    b.d_out = d[1];
    b.last = c == k ? 1 : 0;
    b.bytes = prof ? fused_bytes(c + 1, b.last, true) : 0;
    if (prof) prof_units_ += c;
    launch_cheb_fused(b, s_);
    buf = 1;
    i = c;
    launches++;
  }
  // the remainder of the steps left first, then launches of S steps
  const int i0 = i;
  while (i < k) {
    const int n = i == i0 && (k - i0) % S ? (k - i0) % S : S;
    a.S = n;
    for (int st = 0; st < kFusedMax; st++) a.slots[st] = ops_->fused_slots[n][st];
    for (int s = 0; s < n; s++) {
      a.c1[s] = c1[i + s];
      a.c2[s] = c2[i + s];
    }
    a.d_in = d[buf];
    a.d_out = d[buf ^ 1];
    a.r_in = r[buf];
    a.r_out = r[buf ^ 1];
    a.last = i + n == k ? 1 : 0;
    a.bytes = prof ? fused_bytes(n, a.last, false) : 0;
    if (prof) prof_units_ += n;
    launch_cheb_fused(a, s_);
    buf ^= 1;
    i += n;
    launches++;
  }
  if (prof) bracket_end(launches);
  // partials of r_0.r_0 come from the set-up launch's grid, those of the
  // final residual from the last launch's
  defer_check(1, su ? setup_grid : nwg_init, colK, kneed, su && launches == 1 ? setup_grid : grid);
  stats.solves++;
  stats.cg_iters += k;
  stats.cg_iters_max = std::max(stats.cg_iters_max, k);
}

// Algorithmic bytes of one k_cheb_fused launch of n steps: per row the ELL
// row (5 columns, 5 values), the Jacobi diagonal, x in and out, r and d in,
// r out, d out unless the launch ends the solve, and with n > 1 the row's
// part-local columns (2 bytes each); per part its ring lists for rings
// 1..n-1 (4 bytes a row) and the local columns of rings 1..n-2.  Ring rows'
// own data are other parts' rows, counted once.  A set-up launch reads u
// and the Coriolis row (40 bytes), the row's two cells (8), and x_0's
// addends instead of x, r and d (net +40 bytes a row), and per cell its
// three edges and signs (24), 1/|c| (8), eta (8), two addends (16) and the
// output (8).
unsigned long long Engine::fused_bytes(int n, int last, bool setup) const {
  double b = (double)ne_ * (108.0 + (last ? 0.0 : 8.0) + (n > 1 ? 10.0 : 0.0) + (setup ? 40.0 : 0.0));
  if (setup) b += (double)nc_ * 64.0;
  const pa_ops *o = ops_;
  for (int p = 0; p < o->hparts; p++) {
    const int32_t *c = &o->ring_cnt[(size_t)p * 8];
    b += 32.0;
    if (n >= 2) b += 4.0 * c[n - 2];
    if (n >= 3) b += 10.0 * c[n - 3];
  }
  return (unsigned long long)b;
}

// Steps per fused launch of a single-column solve whose set-up the first
// launch can do (the solve takes the fused Jacobi path), else 0.
int Engine::fused_setup_steps() const {
  if (!cheb() && !mixed()) return 0;
  if (mixed() && 1 >= tune_.mixed_min_cols) return 0;
  if (lp_cheaper(1)) return 0;
  const int S = std::min(tune_.fused_steps, ops_->fused_max);
  if (S < 2 || ops_->fused_cpp <= 0 || cheb_fused_grid(ops_->d) <= 0) return 0;
  return S;
}

void Engine::cheb_solve(double *x, int Bs, const int *colK, int kneed, int nwg_init) {
  const bool lp = lp_cheaper(Bs);
  const int S = std::min(tune_.fused_steps, ops_->fused_max);
  if (!lp && Bs == 1 && S > 1) {
    const int grid = cheb_fused_grid(ops_->d);
    if (grid > 0) return cheb_fused(x, colK, kneed, nwg_init, grid, S, nullptr);
  }
  const std::vector<double> &c1 = lp ? lp_c1_ : cheb_c1_, &c2 = lp ? lp_c2_ : cheb_c2_;
  const int k = (int)c1.size();
  double *d[2] = {p_, s0_};
  if (lp && Bs <= 4) {
    // narrow blocks: one kernel per step, P r_{k+1} = P r_k - (P M) d_k
    LpDirArgs a0{};  // d_0 = theta^-1 P r_0 replaces the set-up kernel's Jacobi direction
    a0.ops = ops_->d;
    a0.lp = ops_->lp;
    a0.Bs = Bs;
    a0.r = r_;
    a0.d_out = d[0];
    a0.c2 = 1.0 / lp_theta_;
    a0.colK = colK;
    a0.kneed = kneed;
    launch_lp_dir(a0, s_);
    ChebLpArgs a{};
    a.ops = ops_->d;
    a.lp = ops_->lp;
    a.Bs = Bs;
    a.x = x;
    a.colK = colK;
    a.kneed = kneed;
    a.part = chk_last_[chk_par_];
    a.max_wg = rb_.max_wg;
    double *r[2] = {r_, r1_};
    const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB_LP_ITER;
    a.prof = prof ? st_.prof : nullptr;
    for (int i = 0; i < k; i++) {
      a.d_in = d[i & 1];
      a.d_out = d[(i + 1) & 1];
      a.r_in = r[i & 1];
      a.r_out = r[(i + 1) & 1];
      a.c1 = c1[i];
      a.c2 = c2[i];
      a.last = i + 1 == k ? 1 : 0;
      if (prof && i == 0) bracket_begin();
      launch_cheb_lp_iter(a, s_);
    }
    if (prof) bracket_end(k);
  } else if (lp) {
    // wide blocks: x and r updated in place by the Jacobi step kernel without
    // its direction, then d_{k+1} = c1 d_k + c2 P r_{k+1} (fewer gathers
    // than the one-kernel form, which also gathers d over P M)
    LpDirArgs b{};
    b.ops = ops_->d;
    b.lp = ops_->lp;
    b.Bs = Bs;
    b.r = r_;
    b.colK = colK;
    b.kneed = kneed;
    b.d_out = d[0];
    b.c1 = 0.0;
    b.c2 = 1.0 / lp_theta_;
    launch_lp_dir(b, s_);
    ChebArgs a{};
    a.ops = ops_->d;
    a.Bs = Bs;
    a.x = x;
    a.r = r_;
    a.colK = colK;
    a.kneed = kneed;
    a.part = chk_last_[chk_par_];
    a.max_wg = rb_.max_wg;
    a.nodir = 1;
    const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB_LP_ITER;
    a.prof = prof ? st_.prof : nullptr;
    for (int i = 0; i < k; i++) {
      a.d_in = d[i & 1];
      a.last = i + 1 == k ? 1 : 0;
      if (prof && i == 0) bracket_begin();
      launch_cheb_iter(a, s_);
      if (!a.last) {
        b.d_in = d[i & 1];
        b.d_out = d[(i + 1) & 1];
        b.c1 = c1[i];
        b.c2 = c2[i];
        launch_lp_dir(b, s_);
      }
    }
    if (prof) bracket_end(2 * k - 1);
  } else if (Bs == 1) {
    // single column, one step per launch (the fused kernel does the same
    // arithmetic several steps at a time)
    ChebArgs a{};
    a.ops = ops_->d;
    a.Bs = Bs;
    a.x = x;
    a.r = r_;
    a.colK = colK;
    a.kneed = kneed;
    a.part = chk_last_[chk_par_];
    a.max_wg = rb_.max_wg;
    const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB_ITER;
    a.prof = prof ? st_.prof : nullptr;
    for (int i = 0; i < k; i++) {
      a.d_in = d[i & 1];
      a.d_out = d[(i + 1) & 1];
      a.c1 = c1[i];
      a.c2 = c2[i];
      a.last = i + 1 == k ? 1 : 0;
      if (prof && i == 0) bracket_begin();
      launch_cheb_iter(a, s_);
    }
    if (prof) bracket_end(k);
  } else {
    // blocks: three-term form on the increment y: y_1 = d_0 (set-up kernel,
    // in p_), k - 1 steps to y_k, then the finishing launch (x += y_k and
    // the residual)
    Cheb3Args a{};
    a.ops = ops_->d;
    a.Bs = Bs;
    a.b = r_;
    a.x = x;
    a.colK = colK;
    a.kneed = kneed;
    a.part = chk_last_[chk_par_];
    a.max_wg = rb_.max_wg;
    const bool prof = ctx_->prof_kernel == PA_KERNEL_CHEB3_ITER;
    a.prof = prof ? st_.prof : nullptr;
    a.prof_bytes = st_.prof_bytes;
    double *cur = d[0], *prev = d[1];
    if (prof) bracket_begin();
    for (int i = 1; i < k; i++) {
      a.y_cur = cur;
      a.y_prev = prev;
      a.y_next = prev;
      a.c1 = c1[i - 1];
      a.c2 = c2[i - 1];
      a.zero_prev = i == 1 ? 1 : 0;
      launch_cheb3_iter(a, s_);
      std::swap(cur, prev);
    }
    a.y_cur = cur;
    a.finish = 1;
    launch_cheb3_iter(a, s_);
    if (prof) bracket_end(k);
  }
  if (lp) stats.precond = PA_PRECOND_LEARNED;
  if (lp) lp_prof_wide_ = Bs > 4;
  stats.lp_solves += lp ? 1 : 0;
  defer_check(Bs, nwg_init, colK, kneed);
  stats.solves++;
  stats.cg_iters += k;
  stats.cg_iters_max = std::max(stats.cg_iters_max, k);
}

void Engine::plan_common(int BsMax) {
  BsMax_ = BsMax;
  const int tiles = tiles_of(BsMax);
  const size_t ebs = (size_t)ne_ * BsMax;
  if (mixed()) {
    r32_ = ar_.take<float>(ebs);
    d32_[0] = ar_.take<float>(ebs);
    d32_[1] = ar_.take<float>(ebs);
  }
  r_ = ar_.take<double>(ebs);   // r[0]; the set-up kernels write r_0 here
  r1_ = ar_.take<double>(ebs);
  w0_ = ar_.take<double>(ebs);
  w1_ = ar_.take<double>(ebs);
  s0_ = ar_.take<double>(ebs);
  s1_ = ar_.take<double>(ebs);
  p_ = ar_.take<double>(ebs);
  st_.bb = ar_.take<double>(BsMax);
  st_.rz = ar_.take<double>(BsMax);
  st_.alpha = ar_.take<double>(BsMax);
  st_.beta = ar_.take<double>(BsMax);
  st_.resid = ar_.take<double>(BsMax);
  st_.active = ar_.take<int>(BsMax);
  st_.iters = ar_.take<int>(BsMax);
  colK0_ = ar_.take<int>(BsMax);
  st_.rz2 = ar_.take<double>(8);
  st_.al2 = ar_.take<double>(8);
  st_.act2 = ar_.take<int>(8);
  st_.it2 = ar_.take<int>(8);
  rb_.max_wg = launch_max_wg();
  rb_.partA = ar_.take<double>((size_t)tiles * rb_.max_wg * 3 * 64);
  rb_.partB = ar_.take<double>((size_t)tiles * rb_.max_wg * 5 * 64);
  // residual partials of Chebyshev solves by solve parity, so that a
  // solve's check can run inside the next solve's set-up kernel
  for (int p = 0; p < 2; p++) {
    chk_init_[p] = ar_.take<double>((size_t)tiles * rb_.max_wg * 64);
    chk_last_[p] = ar_.take<double>((size_t)tiles * rb_.max_wg * 64);
  }
  // counters, cleared at the start of each call
  zero_words_ = 64;
  zero_base_ = ar_.take<unsigned>(zero_words_);
  if (zero_base_) {
    unsigned *z = zero_base_;
    st_.cnt = (int *)z;
    st_.fail = (int *)(z + 2);
    st_.iter_max = (int *)(z + 3);
    st_.prof = z + 4;
    st_.prof_last = z + 6;
    st_.budget_fail = (int *)(z + 7);
    st_.cheb_fail = (int *)(z + 8);
    st_.resid_max = (unsigned long long *)(z + 10);  // 8-byte aligned
    st_.prof_bytes = (unsigned long long *)(z + 12);
  }
}

Blk Engine::block(int Bs) {
  Blk b;
  b.Bs = Bs;
  b.p = ar_.take<double>((size_t)n_ * Bs);
  return b;
}

void Engine::upload(void *dst, const void *src, size_t bytes) {
  if (bytes) PA_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s_));
}

void Engine::begin() {
  if (!ops_->dev) throw Error(PA_EINVAL, "operators are not bound to device memory");
  PA_HIP(hipSetDevice(ctx_->device));
  launch_zero(zero_base_, zero_words_, s_);
  launch_zero((unsigned *)colK0_, BsMax_, s_);
  PA_HIP(hipEventCreate(&ev0_));
  PA_HIP(hipEventCreate(&ev1_));
  PA_HIP(hipEventRecord(ev0_, s_));
  stats = pa_stats{};
  guard_next_ = 0;
  pend_ = false;
  chk_par_ = 0;
}

void Engine::finish() {
  TuneScope tune_scope(tune_);
  PA_HIP(hipEventRecord(ev1_, s_));
  // counters z+2 .. z+11: fail, iter_max, prof[3], budget_fail, cheb_fail,
  // (pad), resid_max bits
  int h[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  PA_HIP(hipMemcpyAsync(h, st_.fail, 12 * sizeof(int), hipMemcpyDeviceToHost, s_));
  sync_checked(s_);
  {
    unsigned long long bits;
    std::memcpy(&bits, &h[8], sizeof(bits));
    double rm;
    std::memcpy(&rm, &bits, sizeof(rm));
    stats.resid_max = rm;
  }
  if (ctx_->prof_kernel != PA_KERNEL_NONE) {
    for (const ProfSpan &p : prof_ev_) {
      float t = 0;
      PA_HIP(hipEventElapsedTime(&t, p.e0, p.e1));
      ctx_->prof_ms += t;
      ctx_->prof_launches += p.n;
      ctx_->prof_pool.push_back(p.e0);
      ctx_->prof_pool.push_back(p.e1);
    }
    prof_ev_.clear();
    // algorithmic bytes: per active column and row, the vectors the kernel
    // must stream once; per row and launch, the matrix row it reads
    const double cols = (unsigned)h[2], work = (unsigned)h[3];
    // x, p, r, w, s in; x, p, r', w', s' out; ELL row (5 cols, 5 values)
    // and the Jacobi diagonal once per launch
    if (ctx_->prof_kernel == PA_KERNEL_CG_ITER)
      ctx_->prof_bytes += (double)ne_ * (80.0 * cols + 68.0 * work);
    // Chebyshev step: x, r, d in; x, r, d' out (d' not on the last step)
    if (ctx_->prof_kernel == PA_KERNEL_CHEB_ITER)
      ctx_->prof_bytes += (double)ne_ * (48.0 * cols + 40.0 * (unsigned)h[4] + 68.0 * work);
    // learned step, per active column and row: x, r, d in and x, r, d' out
    // (d' not on the last step); per row and launch: the mass ELL row and
    // the packed P and P M rows (8 bytes per entry; the wide two-kernel form
    // reads P only, and r and d once more)
    if (ctx_->prof_kernel == PA_KERNEL_CHEB_LP_ITER)
      ctx_->prof_bytes += lp_prof_wide_
                              ? (double)ne_ * (64.0 * cols + 40.0 * (unsigned)h[4] +
                                               (68.0 + 8.0 * ops_->lp_wp) * work)
                              : (double)ne_ * (48.0 * cols + 40.0 * (unsigned)h[4] +
                                               (60.0 + 8.0 * (ops_->lp_wp + ops_->lp_wpm)) * work);
    // fused steps: summed by the kernel from the launches' own figures
    // (fused_bytes)
    if (ctx_->prof_kernel == PA_KERNEL_CHEB_FUSED || ctx_->prof_kernel == PA_KERNEL_CHEB3_ITER ||
        ctx_->prof_kernel == PA_KERNEL_CHEB32_ITER) {
      unsigned long long fb;
      std::memcpy(&fb, &h[10], sizeof(fb));
      ctx_->prof_bytes += (double)fb;
    }
    // mass-solve steps times the columns they ran on: counted on the host
    // for the fused steps (a launch runs several), from the kernels' count
    // of active columns for the one-step kernels
    ctx_->prof_units += ctx_->prof_kernel == PA_KERNEL_CHEB_FUSED ? prof_units_ : cols;
    prof_units_ = 0;
    ctx_->prof_work += (int64_t)work;
  }
  float ms = 0;
  PA_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
  (void)hipEventDestroy(ev0_);
  (void)hipEventDestroy(ev1_);
  ev0_ = ev1_ = nullptr;
  stats.device_ms = ms;
  stats.cg_iters_max = std::max(stats.cg_iters_max, h[1]);
  if (guard_ && guard_bm_ > 0) {
    const int used = std::min(guard_calls_, kGuardSlots);
    std::vector<double> g((size_t)used * 10 * guard_bm_);
    PA_HIP(hipMemcpy(g.data(), guard_, g.size() * sizeof(double), hipMemcpyDeviceToHost));
    const double H = ops_->H, gr = ops_->g;
    for (int sl = 0; sl < used; sl++) {
      const double *q = g.data() + (size_t)sl * 10 * guard_bm_;
      for (int c = 0; c < guard_members_; c++) {
        const double w0 = H * q[c] + gr * q[2 * guard_bm_ + c];
        const double wk = H * q[5 * guard_bm_ + c] + gr * q[7 * guard_bm_ + c];
        if (w0 > 0 && wk > 1.0201 * w0) stats.guard_trips++;  // 1% growth of the norm
      }
    }
    if (stats.guard_trips > 0)
      throw Error(PA_EGROWTH, "Chebyshev basis grows: lambda_bar is below the spectral radius of L");
  }
  if (h[0] > 0)
    throw Error(PA_ENOCONV, std::to_string(h[0]) + " mass-solve column(s) did not converge within maxit");
  if (h[5] > 0) throw BudgetExceeded();
  if (h[6] > 0) throw SolverCheckFailed();
  // next calls on this context run without polling, with this budget
  if (learn_budget_) ctx_->cg_budget[cfg_.cg_rtol] = std::min(cfg_.maxit, h[1] + 2);
}

// Diagnostics of every column of X into out[5][Bs] (see k_diag).
void Engine::diag(Blk X, double *out) {
  DiagArgs d{};
  d.ops = ops_->d;
  d.Bs = X.Bs;
  d.H = ops_->H;
  d.u = X.p;
  d.eta = X.p + (size_t)ne_ * X.Bs;
  d.part = rb_.partB;
  d.max_wg = rb_.max_wg;
  launch_diag(d, s_);
  FinArgs f{};
  f.mode = FIN_OUT;
  f.Bs = X.Bs;
  f.nwg = launch_rows_grid(std::max(ne_, nc_), X.Bs);
  f.max_wg = rb_.max_wg;
  f.nq = 5;
  f.part = rb_.partB;
  f.st = st_;
  f.out = out;
  launch_finalize(f, s_);
}

// Measurement hook.  The steps of one mass solve are launched back to back
// with nothing between them, so one event pair around the sequence times n
// launches (kernel time plus the dispatch gaps between them); events around
// each launch would add their own overhead to every launch.  CG iterations
// alternate with other kernels and are timed one by one with events that
// the dispatch itself records (arm_events).
void Engine::bracket_begin() {
  ProfSpan p;
  p.e0 = take_event();
  p.e1 = take_event();
  PA_HIP(hipEventRecord(p.e0, s_));
  prof_ev_.push_back(p);
}

void Engine::bracket_end(int n) {
  ProfSpan &p = prof_ev_.back();
  PA_HIP(hipEventRecord(p.e1, s_));
  p.n = n;
}

void Engine::arm_events() {
  ProfSpan p;
  p.e0 = take_event();
  p.e1 = take_event();
  p.n = 1;
  arm_launch_events(p.e0, p.e1);
  prof_ev_.push_back(p);
}

hipEvent_t Engine::take_event() {
  if (!ctx_->prof_pool.empty()) {
    hipEvent_t e = ctx_->prof_pool.back();
    ctx_->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PA_HIP(hipEventCreate(&e));
  return e;
}

void Engine::axpy(size_t n, double *out, double a0, const double *x0, double a1, const double *x1,
                  double a2, const double *x2) {
  AxpyArgs a{n, a0, a1, a2, x0, x1, x2, out};
  launch_axpy(a, s_);
}

// Batched CG on the velocity mass matrix for the columns the preceding
// set-up kernel prepared (r_0 in r[0], start value in x).  Convergence is
// decided per column on the device.  Small batches (Bs <= 4) run the fused
// kernels (one launch per iteration, each workgroup reducing the previous
// partials); larger ones follow each iteration with a finalize kernel.
// Without an iteration budget the host polls the active count (first after
// the predicted count); with one (learned from earlier calls on the context)
// exactly that many iterations are launched and convergence is checked once
// at the end of the call.
void Engine::cg(double *x, int Bs, const int *colK, int kneed, int nwg_init) {
  (void)nwg_init;
  CgArgs a{};
  a.ops = ops_->d;
  a.Bs = Bs;
  a.x = x;
  a.p = p_;
  a.rtol2 = cfg_.cg_rtol * cfg_.cg_rtol;
  a.maxit = cfg_.maxit;
  a.st = st_;
  a.rb = rb_;
  a.count_cols = ctx_->prof_kernel == PA_KERNEL_CG_ITER ? 1 : 0;
  a.colK = colK;
  a.kneed = kneed;
  const int nwg = launch_rows_grid(ne_, Bs);
  int budget = 0;
  if (budget_ok_) {
    auto itb = ctx_->cg_budget.find(cfg_.cg_rtol);
    if (itb != ctx_->cg_budget.end()) budget = itb->second;
  }
  double *r[2] = {r_, r1_}, *w[2] = {w0_, w1_}, *sv[2] = {s0_, s1_};
  double *part[2] = {rb_.partA, rb_.partB};
  int *hflag = (int *)ctx_->host_flag;
  auto timed = [&](auto launch) {
    if (ctx_->prof_kernel == PA_KERNEL_CG_ITER) arm_events();
    launch();
  };
  auto poll = [&](int slot) {
    PA_HIP(hipMemcpyAsync(hflag, st_.cnt + slot, sizeof(int), hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    return *hflag;
  };
  // w_0 = M D^-1 r_0 and the first partials
  a.r_in = r[0];
  a.w_out = w[0];
  a.part_out = part[0];
  launch_cg_init(a, s_);
  // iteration k reads r[k&1], w[k&1], s[(k+1)&1]; writes the other halves
  auto iter = [&](int k, bool last) {
    a.k = k;
    a.r_in = r[k & 1];
    a.r_out = r[(k + 1) & 1];
    a.w_in = w[k & 1];
    a.w_out = w[(k + 1) & 1];
    a.s_in = sv[(k + 1) & 1];
    a.s_out = sv[k & 1];
    a.part_in = part[k & 1];
    a.part_out = part[(k + 1) & 1];
    a.nwg_prev = nwg;
    a.last_check = last ? 1 : 0;
    a.check_only = last ? 1 : 0;
    timed([&] { launch_cg_iter(a, s_); });
  };
  int it = 0;
  if (Bs <= 4) {
    // kernel k tests r_k and, if needed, performs iteration k
    a.fused = 1;
    if (budget > 0) {
      for (int k = 0; k <= budget; k++) iter(k, k == budget);
      it = budget;
    } else {
      int chunk = std::max(1, std::min(predicted_, cfg_.maxit)) + 1;
      for (;;) {
        for (int i = 0; i < chunk && it <= cfg_.maxit; i++) iter(it++, false);
        if (poll((it - 1) & 1) == 0 || it > cfg_.maxit) break;
        chunk = 1;
      }
      it -= 1;
    }
  } else {
    // kernel k performs iteration k; the finalize after it tests r_{k+1}
    a.fused = 0;
    FinArgs fa{};
    fa.Bs = Bs;
    fa.max_wg = rb_.max_wg;
    fa.nq = 3;
    fa.st = st_;
    fa.rtol2 = a.rtol2;
    fa.maxit = a.maxit;
    fa.mode = FIN_INIT;
    fa.nwg = nwg;
    fa.part = part[0];
    fa.colK = colK;
    fa.kneed = kneed;
    fa.slot_out = 1;
    launch_finalize(fa, s_);
    fa.mode = FIN_STEP;
    const int total = budget > 0 ? budget : cfg_.maxit;
    int chunk = budget > 0 ? budget : std::max(1, std::min(predicted_, cfg_.maxit));
    for (;;) {
      for (int i = 0; i < chunk && it < total; i++) {
        const int k = it++;
        iter(k, false);
        fa.part = part[(k + 1) & 1];
        fa.slot_in = (k + 1) & 1;
        fa.slot_out = k & 1;
        fa.last_check = (budget > 0 && it == budget) ? 1 : 0;
        launch_finalize(fa, s_);
      }
      if (budget > 0 || it >= total) break;
      if (poll((it - 1) & 1) == 0) break;
      chunk = 1;
    }
  }
  predicted_ = std::max(1, it - 1);
  stats.solves++;
  stats.cg_iters += it;
  stats.budget = budget;
}

void Engine::lstep(Blk in, Blk out, const Blk *A, const Blk *B, double scale, const int *colK,
                   int kneed, const AccSpec *acc) {
  StiffArgs a{};
  a.ops = ops_->d;
  a.Bs = in.Bs;
  a.in_u = in.p;
  a.in_eta = in.p + (size_t)ne_ * in.Bs;
  a.out_u = out.p;
  a.out_eta = out.p + (size_t)ne_ * in.Bs;
  if (A) {
    a.addA_u = A->p;
    a.addA_eta = A->p + (size_t)ne_ * in.Bs;
  }
  if (B) {
    a.addB_u = B->p;
    a.addB_eta = B->p + (size_t)ne_ * in.Bs;
  }
  a.scale = scale;
  a.colK = colK;
  a.kneed = kneed;
  a.r = r_;
  if (acc) {
    a.acc_u = acc->acc;
    a.acc_eta = acc->acc + (size_t)ne_ * (in.Bs / acc->G);
    a.coef = acc->coef;
    a.acc_k = acc->acc_k;
    a.G = acc->G;
  } else {
    a.G = 1;
  }
  a.st = st_;
  a.rb = rb_;
  a.max_wg = rb_.max_wg;
  // a single-column Jacobi Chebyshev solve folds this set-up into its first
  // fused launch
  const int S = acc || in.Bs != 1 ? 0 : fused_setup_steps();
  if (S > 0) {
    const FusedSetup su{a.in_u, a.in_eta, a.addA_u, a.addA_eta, a.addB_u, a.addB_eta, a.out_eta, scale};
    const int grid = cheb_fused_grid(ops_->d);
    cheb_fused(out.p, colK, kneed, grid, grid, S, &su);
    return;
  }
  if (cheb() || mixed()) {
    a.d0 = p_;
    a.theta_inv = 1.0 / cheb_theta_;
    a.part_rr = chk_init_[chk_par_];
    take_check(a.chk, a.chk_blocks,
               launch_rows_grid(std::max(ne_, nc_), in.Bs) * tiles_of(in.Bs));
  }
  launch_stiff(a, s_);
  mass_solve(out.p, in.Bs, colK, kneed, launch_rows_grid(std::max(ne_, nc_), in.Bs));
}

// acc = sum_k coef_k (.) R_k(X) over the real Chebyshev recurrence, with the
// per-degree sums fused into the next step's operator application; grouped
// over G columns when G > 1.  X and W are overwritten.
void Engine::poly_apply(Blk X, Blk W, const double *coef, const int *colK, int kmax, int G,
                        Blk acc) {
  const int Bs = X.Bs;
  const double lb = ops_->lambda_bar;
  axpy((size_t)n_ * acc.Bs, acc.p, 0.0, nullptr);
  auto acc_only = [&](Blk R, int k) {
    AccArgs a{n_, Bs, G, k, R.p, coef + (size_t)k * Bs, colK, acc.p};
    launch_acc(a, s_);
  };
  if (kmax == 0) {
    acc_only(X, 0);
    return;
  }
  AccSpec as;
  as.acc = acc.p;
  as.G = G;
  as.coef = coef;
  as.acc_k = 0;
  lstep(X, W, nullptr, nullptr, 1.0 / lb, colK, 1, &as);
  Blk prev = X, cur = W;
  for (int k = 1; k < kmax; k++) {
    as.coef = coef + (size_t)k * Bs;
    as.acc_k = k;
    lstep(cur, prev, &prev, nullptr, 2.0 / lb, colK, k + 1, &as);
    std::swap(prev, cur);
  }
  acc_only(cur, kmax);
  stats.kmax = std::max(stats.kmax, kmax);
}

// N of every column of E into Y (columns with colK >= 0).
void Engine::nonlinear_block(Blk E, Blk Y, const int *colK) {
  NlArgs a{};
  a.ops = ops_->d;
  a.Bs = E.Bs;
  a.u = E.p;
  a.eta = E.p + (size_t)ne_ * E.Bs;
  a.C = C_;
  a.out_eta = Y.p + (size_t)ne_ * E.Bs;
  launch_nl_cell(a, s_);
  GatherArgs gth{};
  gth.ops = ops_->d;
  gth.Bs = E.Bs;
  gth.C = C_;
  gth.r = r_;
  gth.x = Y.p;
  gth.colK = colK;
  gth.kneed = 0;
  gth.st = st_;
  gth.rb = rb_;
  gth.max_wg = rb_.max_wg;
  const bool refined = mixed() && E.Bs >= tune_.mixed_min_cols;
  if (cheb() || mixed()) {
    if (refined) {
      // the gather writes the first refinement's outputs
      gth.r32 = r32_;
      gth.x1_32 = d32_[0];
      gth.theta_inv32 = (float)(1.0 / cheb_theta_);
    } else {
      gth.d0 = p_;
      gth.theta_inv = 1.0 / cheb_theta_;
    }
    gth.part_rr = chk_init_[chk_par_];
    take_check(gth.chk, gth.chk_blocks, launch_rows_grid(ne_, E.Bs) * tiles_of(E.Bs));
  }
  launch_nl_gather(gth, s_);
  if (refined)
    mixed_solve(Y.p, E.Bs, colK, 0, launch_rows_grid(ne_, E.Bs), true);
  else
    mass_solve(Y.p, E.Bs, colK, 0, launch_rows_grid(ne_, E.Bs));
}

// ------------------------------------------------------------- exponential
void Engine::plan_exp(ExpBufs &eb, int B, const double *t) {
  eb.Bs = pad_cols(B);
  const double lb = ops_->lambda_bar;
  std::vector<std::vector<double>> cs(B);
  eb.kmax = 0;
  eb.hcolK.assign(eb.Bs, -1);
  for (int j = 0; j < B; j++) {
    const double th = lb * std::fabs(t[j]);
    const int kcap = 2 * (int)std::ceil(th) + 64;
    cs[j] = bessel_weights(th, kcap);
    const int K = t[j] == 0.0 ? 0 : truncate_degree(cs[j], cfg_.cheb_tol);
    eb.hcolK[j] = K;
    eb.kmax = std::max(eb.kmax, K);
  }
  eb.hcoef.assign((size_t)(eb.kmax + 1) * eb.Bs, 0.0);
  for (int j = 0; j < B; j++) {
    const double sg = t[j] < 0 ? -1.0 : 1.0;
    double sk = 1.0;
    for (int k = 0; k <= eb.hcolK[j]; k++, sk *= sg) eb.hcoef[(size_t)k * eb.Bs + j] = cs[j][k] * sk;
  }
  eb.X = ar_.take<double>((size_t)n_ * eb.Bs);
  eb.W = ar_.take<double>((size_t)n_ * eb.Bs);
  // room for degrees up to 255 so that sizing with one time step covers others
  eb.coef = ar_.take<double>(std::max<size_t>(eb.hcoef.size(), (size_t)256 * eb.Bs));
  eb.colK = ar_.take<int>(eb.Bs);
}

void Engine::run_exp(ExpBufs &eb, Blk in, Blk out) {
  upload(eb.coef, eb.hcoef.data(), eb.hcoef.size() * sizeof(double));
  upload(eb.colK, eb.hcolK.data(), eb.hcolK.size() * sizeof(int));
  axpy((size_t)n_ * eb.Bs, eb.X, 1.0, in.p);
  poly_apply(Blk{eb.X, eb.Bs}, Blk{eb.W, eb.Bs}, eb.coef, eb.colK, eb.kmax, 1, out);
}

void Engine::expL_apply(int B, const double *t, const double *Uin, double *Uout) {
  TuneScope tune_scope(tune_);
  if (B <= 0) throw Error(PA_EINVAL, "B must be positive");
  if (!(ops_->lambda_bar > 0)) throw Error(PA_EINVAL, "lambda_bar is not set");
  if (cfg_.exponential == PA_EXP_REXI) return rexi_expL_apply(B, t, Uin, Uout);
  const int Bs = pad_cols(B);
  plan_common(Bs);
  ExpBufs eb;
  plan_exp(eb, B, t);
  C_ = nullptr;
  Blk in = block(Bs), out = block(Bs);
  if (ar_.sizing()) return;
  begin();
  TransArgs tr{n_, B, Bs, const_cast<double *>(Uin), in.p};
  launch_to_block(tr, s_);
  run_exp(eb, in, out);
  flush_check();
  TransArgs tb{n_, B, Bs, Uout, out.p};
  launch_from_block(tb, s_);
  finish();
}

// ---------------------------------------------------------- nonlinearity
void Engine::swe_nonlinear(int B, const double *U, double *NU) {
  TuneScope tune_scope(tune_);
  if (B <= 0) throw Error(PA_EINVAL, "B must be positive");
  const int Bs = pad_cols(B);
  plan_common(Bs);
  C_ = ar_.take<double>((size_t)3 * nc_ * Bs);
  int *colK = ar_.take<int>(Bs);
  Blk E = block(Bs), Y = block(Bs);
  if (ar_.sizing()) return;
  begin();
  std::vector<int> hk(Bs, -1);
  for (int j = 0; j < B; j++) hk[j] = 0;
  upload(colK, hk.data(), hk.size() * sizeof(int));
  TransArgs tr{n_, B, Bs, const_cast<double *>(U), E.p};
  launch_to_block(tr, s_);
  nonlinear_block(E, Y, colK);
  flush_check();
  TransArgs tb{n_, B, Bs, NU, Y.p};
  launch_from_block(tb, s_);
  finish();
}

// ------------------------------------------------------ averaged RHS
void Engine::plan_nbar(NbarBufs &nb, const pa_avg *avg, int members) {
  const double lb = ops_->lambda_bar;
  if (!(lb > 0)) throw Error(PA_EINVAL, "lambda_bar is not set");
  // terms kept: weights above the cut
  double wmax = 0;
  for (double w : avg->w) wmax = std::max(wmax, std::fabs(w));
  std::vector<int> keep;
  for (size_t m = 0; m < avg->w.size(); m++)
    if (std::fabs(avg->w[m]) >= cfg_.weight_cut * wmax && avg->w[m] != 0.0) keep.push_back((int)m);
  nb.M = (int)keep.size();
  if (nb.M == 0) throw Error(PA_EINVAL, "no averaging terms");
  if (nb.M > 64) throw Error(PA_ENOTSUP, "at most 64 averaging terms per call");
  nb.members = members;
  nb.Bm = pad_cols(members);
  nb.G = pad_cols(nb.M);
  nb.BsE = nb.Bm * nb.G;
  std::vector<std::vector<double>> cs(nb.M);
  std::vector<int> K(nb.M);
  nb.kmax = 0;
  nb.ksum = 0;
  for (int i = 0; i < nb.M; i++) {
    const double s = avg->s[keep[i]];
    const double th = lb * std::fabs(s);
    cs[i] = bessel_weights(th, 2 * (int)std::ceil(th) + 64);
    K[i] = s == 0.0 ? 0 : truncate_degree(cs[i], cfg_.cheb_tol);
    nb.kmax = std::max(nb.kmax, K[i]);
    nb.ksum += K[i];
  }
  const int G = nb.G, kmax = nb.kmax;
  nb.hcF.assign((size_t)(kmax + 1) * G, 0.0);
  nb.hcB.assign((size_t)(kmax + 1) * G, 0.0);
  for (int i = 0; i < nb.M; i++) {
    const double s = avg->s[keep[i]], w = avg->w[keep[i]];
    double sf = 1.0, sb = 1.0;
    const double gf = s < 0 ? -1.0 : 1.0;
    for (int k = 0; k <= K[i]; k++, sf *= gf, sb *= -gf) {
      nb.hcF[(size_t)k * G + i] = cs[i][k] * sf;
      nb.hcB[(size_t)k * G + i] = w * cs[i][k] * sb;
    }
  }
  nb.hcBx.assign((size_t)(kmax + 1) * nb.BsE, 0.0);
  nb.hcolK_E.assign(nb.BsE, -1);
  for (int mem = 0; mem < members; mem++)
    for (int i = 0; i < nb.M; i++) {
      const int c = mem * G + i;
      nb.hcolK_E[c] = K[i];
      for (int k = 0; k <= kmax; k++) nb.hcBx[(size_t)k * nb.BsE + c] = nb.hcB[(size_t)k * G + i];
    }
  nb.hcolK_fwd.assign(nb.Bm, -1);
  nb.hcolK_mem.assign(nb.Bm, -1);
  for (int mem = 0; mem < members; mem++) {
    nb.hcolK_fwd[mem] = kmax;
    nb.hcolK_mem[mem] = 0;
  }
  const size_t blkm = (size_t)n_ * nb.Bm, blke = (size_t)n_ * nb.BsE;
  nb.basis = ar_.take<double>((size_t)(kmax + 1) * blkm);
  nb.E = ar_.take<double>(blke);
  nb.Y = ar_.take<double>(blke);
  nb.W = ar_.take<double>(blke);
  if (cfg_.backward == PA_BACKWARD_CLENSHAW) {
    nb.Z = ar_.take<double>((size_t)(kmax + 1) * blkm);
    nb.b1 = ar_.take<double>(blkm);
    nb.b2 = ar_.take<double>(blkm);
  }
  nb.cF = ar_.take<double>(nb.hcF.size());
  nb.cB = ar_.take<double>(nb.hcB.size());
  nb.cBx = ar_.take<double>(nb.hcBx.size());
  nb.colK_E = ar_.take<int>(nb.BsE);
  nb.colK_fwd = ar_.take<int>(nb.Bm);
  nb.colK_mem = ar_.take<int>(nb.Bm);
}

void Engine::upload_nbar(NbarBufs &nb) {
  upload(nb.cF, nb.hcF.data(), nb.hcF.size() * sizeof(double));
  upload(nb.cB, nb.hcB.data(), nb.hcB.size() * sizeof(double));
  upload(nb.cBx, nb.hcBx.data(), nb.hcBx.size() * sizeof(double));
  upload(nb.colK_E, nb.hcolK_E.data(), nb.hcolK_E.size() * sizeof(int));
  upload(nb.colK_fwd, nb.hcolK_fwd.data(), nb.hcolK_fwd.size() * sizeof(int));
  upload(nb.colK_mem, nb.hcolK_mem.data(), nb.hcolK_mem.size() * sizeof(int));
}

void Engine::run_nbar(NbarBufs &nb, Blk X, Blk out, bool uploaded) {
  const double lb = ops_->lambda_bar;
  if (!uploaded) upload_nbar(nb);
  const int Bm = nb.Bm, kmax = nb.kmax;
  const size_t blkm = (size_t)n_ * Bm;
  auto R = [&](int k) { return Blk{nb.basis + (size_t)k * blkm, Bm}; };
  // forward basis R_0..R_kmax of the member states (X may already be R_0)
  if (X.p != R(0).p) axpy(blkm, R(0).p, 1.0, X.p);
  if (kmax >= 1) {
    Blk r1 = R(1);
    lstep(R(0), r1, nullptr, nullptr, 1.0 / lb, nb.colK_fwd, 1, nullptr);
  }
  for (int k = 1; k < kmax; k++) {
    Blk rm = R(k - 1);
    lstep(R(k), R(k + 1), &rm, nullptr, 2.0 / lb, nb.colK_fwd, k + 1, nullptr);
  }
  // growth guard: with lambda_bar >= rho(L) every R_k = i^k T_k(-iL/lambda_bar) U
  // has W-norm at most that of U (T_k is bounded by 1 on the real spectrum of
  // -iL/lambda_bar); an underestimated lambda_bar makes the outer modes grow
  if (guard_) {
    double *slot = guard_ + (size_t)std::min(guard_next_++, kGuardSlots - 1) * 10 * Bm;
    diag(R(0), slot);
    diag(R(kmax), slot + 5 * (size_t)Bm);
  }
  // shifted states E[:, mem*G + m] = sum_k cF[k][m] R_k[:, mem]
  CombineArgs ca{n_, nb.BsE, Bm, nb.G, nb.members, kmax, blkm, nb.basis, nb.cF, nb.E};
  launch_combine(ca, s_);
  // N of every shifted state
  nonlinear_block(Blk{nb.E, nb.BsE}, Blk{nb.Y, nb.BsE}, nb.colK_E);
  stats.terms += nb.M * nb.members;
  stats.ksum += nb.ksum * nb.members;
  stats.kmax = std::max(stats.kmax, kmax);
  if (cfg_.backward == PA_BACKWARD_CLENSHAW) {
    // Z_k = sum_m w_m c_k(-s_m) Y_m, then one Clenshaw recurrence per member:
    // b_k = Z_k + (2/lb) L b_{k+1} + b_{k+2}; result Z_0 + L b_1 / lb + b_2.
    ReduceTermsArgs ra{n_, nb.BsE, Bm, nb.G, kmax, blkm, nb.Y, nb.cB, nb.Z};
    launch_reduce_terms(ra, s_);
    auto Z = [&](int k) { return Blk{nb.Z + (size_t)k * blkm, Bm}; };
    if (kmax == 0) {
      axpy(blkm, out.p, 1.0, Z(0).p);
    } else {
      // b_{k+1}, b_{k+2}; b_kmax is Z_kmax itself, whose storage then takes
      // b_{kmax-2}, ... in turn with b2 (no copy)
      Blk bk1 = Z(kmax), bk2{nb.b2, Bm};
      bool have2 = false;
      for (int k = kmax - 1; k >= 1; k--) {
        Blk zk = Z(k);
        // b_k overwrites b_{k+2}
        lstep(bk1, bk2, &zk, have2 ? &bk2 : nullptr, 2.0 / lb, nb.colK_mem, 0, nullptr);
        std::swap(bk1, bk2);
        have2 = true;
      }
      Blk z0 = Z(0);
      lstep(bk1, out, &z0, have2 ? &bk2 : nullptr, 1.0 / lb, nb.colK_mem, 0, nullptr);
    }
  } else {
    // per-term backward recurrences with the weighted sum over terms fused
    poly_apply(Blk{nb.Y, nb.BsE}, Blk{nb.W, nb.BsE}, nb.cBx, nb.colK_E, kmax, nb.G, out);
  }
}

void Engine::nbar_plan(NbarCall &c, const pa_avg *avg, int members, const double *U,
                       double *Nbar) {
  TuneScope tune_scope(tune_);
  if (members <= 0) throw Error(PA_EINVAL, "members must be positive");
  c.avg = avg;
  c.members = members;
  c.U = U;
  c.Nbar = Nbar;
  plan_nbar(c.nb, avg, members);  // sizes first (needs G, BsE)
  plan_common(c.nb.BsE);
  if (cfg_.growth_guard) {
    guard_ = ar_.take<double>((size_t)kGuardSlots * 10 * c.nb.Bm);
    guard_bm_ = c.nb.Bm;
    guard_members_ = members;
    guard_calls_ = 1;
  }
  C_ = ar_.take<double>((size_t)3 * nc_ * c.nb.BsE);
  c.out = block(c.nb.Bm);
}

void Engine::nbar_begin(NbarCall &c) {
  TuneScope tune_scope(tune_);
  begin();
  upload_nbar(c.nb);
}

void Engine::nbar_body(NbarCall &c) {
  TuneScope tune_scope(tune_);
  // the members go straight into R_0 of the basis; with one member the block
  // layout is the state layout, and the result is formed in place
  const Blk r0{c.nb.basis, c.nb.Bm};
  TransArgs tr{n_, c.members, c.nb.Bm, const_cast<double *>(c.U), r0.p};
  launch_to_block(tr, s_);
  const bool direct = c.members == 1 && c.nb.Bm == 1;
  run_nbar(c.nb, r0, direct ? Blk{c.Nbar, 1} : c.out, true);
  flush_check();
  if (!direct) {
    TransArgs tb{n_, c.members, c.nb.Bm, c.Nbar, c.out.p};
    launch_from_block(tb, s_);
  }
}

// A call is a fixed kernel sequence with no host synchronisation when the
// mass solves need no polling (Chebyshev, mixed, or a known CG budget).
int Engine::current_budget() const {
  if (!budget_ok_) return 0;
  auto itb = ctx_->cg_budget.find(cfg_.cg_rtol);
  return itb != ctx_->cg_budget.end() ? itb->second : 0;
}

bool Engine::sync_free() const { return current_budget() > 0 || cheb() || mixed(); }

void Engine::phase_avg_rhs(const pa_avg *avg, int members, const double *U, double *Nbar) {
  TuneScope tune_scope(tune_);
  if (cfg_.exponential == PA_EXP_REXI) return rexi_phase_avg_rhs(avg, members, U, Nbar);
  NbarCall c;
  nbar_plan(c, avg, members, U, Nbar);
  if (ar_.sizing()) return;
  nbar_begin(c);
  // Graph replay: a sync-free call is captured once (on the context's own
  // capture stream) and replayed while nothing it depends on changes.
  if (cfg_.use_graph && sync_free() && ctx_->prof_kernel == PA_KERNEL_NONE) {
    GraphKey key;
    key.ops_gen = ops_->gen;
    key.avg_gen = avg->gen;
    key.members = members;
    key.in = U;
    key.out = Nbar;
    key.ws = ws_base_;
    key.budget = current_budget();
    key.lambda_bar = ops_->lambda_bar;
    key.cfg = cfg_;
    key.tune = tune_;
    run_graph(key, [&] { nbar_body(c); });
  } else {
    nbar_body(c);
  }
  finish();
}

// Capture 'body' into a graph (or reuse the context's graph for the same
// key) and launch it, ordered after the work already on the caller's stream.
void Engine::run_graph(const GraphKey &key, const std::function<void()> &body) {
  if (!ctx_->cap_stream) PA_HIP(hipStreamCreateWithFlags(&ctx_->cap_stream, hipStreamNonBlocking));
  if (!ctx_->ev_a) PA_HIP(hipEventCreateWithFlags(&ctx_->ev_a, hipEventDisableTiming));
  if (!ctx_->ev_b) PA_HIP(hipEventCreateWithFlags(&ctx_->ev_b, hipEventDisableTiming));
  hipStream_t caller = s_, cs = ctx_->cap_stream;
  PA_HIP(hipEventRecord(ctx_->ev_a, caller));
  PA_HIP(hipStreamWaitEvent(cs, ctx_->ev_a, 0));
  if (!(ctx_->graph_exec && ctx_->graph_key == key)) {
    if (ctx_->graph_exec) (void)hipGraphExecDestroy(ctx_->graph_exec);
    ctx_->graph_exec = nullptr;
    hipGraph_t g = nullptr;
    s_ = cs;
    PA_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      body();
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      s_ = caller;
      throw;
    }
    PA_HIP(hipStreamEndCapture(cs, &g));
    s_ = caller;
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw Error(PA_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    ctx_->graph_exec = ex;
    ctx_->graph_key = key;
    ctx_->graph_stats = stats;
    stats.graph_captured = 1;
  } else {
    stats = ctx_->graph_stats;
  }
  PA_HIP(hipGraphLaunch(ctx_->graph_exec, cs));
  PA_HIP(hipEventRecord(ctx_->ev_b, cs));
  PA_HIP(hipStreamWaitEvent(caller, ctx_->ev_b, 0));
  stats.graph = 1;
}

// ---------------------------------------------------------------- RK4 step
// Stages of the averaged Lawson scheme (Sec. 2.3), written for U:
//   k1 = Nbar(U);                U1 = U + dt/2 k1
//   k2 = Nbar(exp(L dt/2) U1);   U2 = exp(L dt/2) U + dt/2 k2
//   k3 = Nbar(U2);               U3 = exp(L dt/2) U + dt k3
//   k4 = Nbar(exp(L dt/2) U3)
//   U+ = exp(L dt)(U + dt/6 k1) + exp(L dt/2)(dt/3 (k2 + k3)) + dt/6 k4
// (exp(L dt/2) exp(L s) = exp(L s) exp(L dt/2) as polynomials in L, and the
// exponentials are linear, so the printed stage-4 sum regroups this way).
void Engine::step(const pa_avg *avg, double dt, int members, double *U) {
  TuneScope tune_scope(tune_);
  if (cfg_.exponential == PA_EXP_REXI) return rexi_step(avg, dt, members, U);
  if (members <= 0) throw Error(PA_EINVAL, "members must be positive");
  NbarBufs nb;
  plan_nbar(nb, avg, members);
  const int Bm = nb.Bm;
  plan_common(nb.BsE);
  if (cfg_.growth_guard) {  // the four averaged right-hand sides of a step
    guard_ = ar_.take<double>((size_t)kGuardSlots * 10 * nb.Bm);
    guard_bm_ = nb.Bm;
    guard_members_ = members;
    guard_calls_ = 4;
  }
  C_ = ar_.take<double>((size_t)3 * nc_ * nb.BsE);
  std::vector<double> th(members, 0.5 * dt), tf(members, dt);
  ExpBufs eh, ef;
  plan_exp(eh, members, th.data());
  plan_exp(ef, members, tf.data());
  Blk X = block(Bm), k1 = block(Bm), k2 = block(Bm), k3 = block(Bm), k4 = block(Bm);
  Blk Eh = block(Bm), T = block(Bm), S = block(Bm);
  if (ar_.sizing()) return;
  begin();
  const size_t nb_ = (size_t)n_ * Bm;
  TransArgs tr{n_, members, Bm, U, X.p};
  launch_to_block(tr, s_);
  upload_nbar(nb);
  run_nbar(nb, X, k1, true);
  axpy(nb_, T.p, 1.0, X.p, 0.5 * dt, k1.p);  // U1
  run_exp(eh, T, S);                          // exp(L dt/2) U1
  run_nbar(nb, S, k2, true);
  run_exp(eh, X, Eh);                         // exp(L dt/2) U
  axpy(nb_, T.p, 1.0, Eh.p, 0.5 * dt, k2.p);  // U2
  run_nbar(nb, T, k3, true);
  axpy(nb_, T.p, 1.0, Eh.p, dt, k3.p);        // U3
  run_exp(eh, T, S);
  run_nbar(nb, S, k4, true);
  axpy(nb_, T.p, 1.0, X.p, dt / 6.0, k1.p);
  run_exp(ef, T, S);                          // exp(L dt)(U + dt/6 k1)
  axpy(nb_, T.p, dt / 3.0, k2.p, dt / 3.0, k3.p);
  run_exp(eh, T, Eh);                         // exp(L dt/2)(dt/3 (k2 + k3))
  axpy(nb_, X.p, 1.0, S.p, 1.0, Eh.p, dt / 6.0, k4.p);
  flush_check();
  TransArgs tb{n_, members, Bm, U, X.p};
  launch_from_block(tb, s_);
  finish();
}

// ------------------------------------------------------------ lambda_bar
double Engine::estimate_lambda(int iters) {
  TuneScope tune_scope(tune_);
  plan_common(1);
  Blk v = block(1), a = block(1), b = block(1);
  double *wd = ar_.take<double>(5);
  if (ar_.sizing()) return 0.0;
  begin();
  // start vector from a counter hash (SplitMix64 of the index), in [-1, 1)
  std::vector<double> h(n_);
  for (int i = 0; i < n_; i++) {
    uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    h[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  upload(v.p, h.data(), sizeof(double) * n_);
  auto wnorm2 = [&](Blk x) {
    diag(x, wd);
    double hv[5];
    PA_HIP(hipMemcpyAsync(hv, wd, 5 * sizeof(double), hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    return ops_->H * hv[0] + ops_->g * hv[2];
  };
  double rho2 = 0.0;
  for (int it = 0; it < iters; it++) {
    const double nv = std::sqrt(wnorm2(v));
    axpy(n_, v.p, 1.0 / nv, v.p);
    lstep(v, a, nullptr, nullptr, 1.0, colK0_, 0, nullptr);  // a = L v
    rho2 = wnorm2(a);                                         // <v,-L^2 v>_W
    lstep(a, b, nullptr, nullptr, 1.0, colK0_, 0, nullptr);  // b = L a
    axpy(n_, v.p, -1.0, b.p);
  }
  flush_check();
  finish();
  return std::sqrt(rho2);
}

void Engine::diagnostics(int B, const double *U, double *out_host) {
  TuneScope tune_scope(tune_);
  const int Bs = pad_cols(B);
  plan_common(Bs);
  Blk X = block(Bs);
  double *wd = ar_.take<double>(5 * (size_t)Bs);
  if (ar_.sizing()) return;
  begin();
  TransArgs tr{n_, B, Bs, const_cast<double *>(U), X.p};
  launch_to_block(tr, s_);
  diag(X, wd);
  std::vector<double> h(5 * (size_t)Bs);
  PA_HIP(hipMemcpyAsync(h.data(), wd, h.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
  finish();
  const double H = ops_->H, g = ops_->g;
  for (int j = 0; j < B; j++) {
    const double uMu = h[j], mass = h[Bs + j], e2 = h[2 * Bs + j], div2 = h[3 * Bs + j];
    const double ke = h[4 * Bs + j];
    out_host[5 * j + 0] = mass;
    out_host[5 * j + 1] = 0.5 * (H * uMu + g * e2);
    out_host[5 * j + 2] = ke + 0.5 * g * e2;
    out_host[5 * j + 3] = std::sqrt(uMu + div2);
    out_host[5 * j + 4] = std::sqrt(e2);
  }
}

}  // namespace pa
