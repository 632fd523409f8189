// Rational (REXI) exponential of libpa: the poles and coefficients of the
// rational sum, the batched shifted solves, and the exponential, the
// averaged right-hand side and the RK4 step built on them.
//
// The rational function is the N-point trapezoidal rule of the Cauchy
// integral of exp(i theta x) over the ellipse X(phi) = cosh(eta0 + i phi)
// around [-1, 1] (Trefethen and Weideman, SIAM Review 56, 2014):
//   exp(i theta x) ~ sum_j c_j / (X_j - x),  c_j = exp(i theta X_j) W_j,
//   X_j = cosh(eta0 + i phi_j),  W_j = sinh(eta0 + i phi_j) / N,
//   phi_j = 2 pi (j + 1/2) / N.
// With x the spectrum of -iL/lb (in [-1, 1] when lb >= rho(L)) and
// theta = lb t this is exp(t L) = sum_j c_j (X_j + (i/lb) L)^-1.  For N a
// multiple of 4 the node phi_j pairs with pi - phi_j (X -> -conj X) and their
// terms are complex conjugates, so the P = N/2 nodes with phi in
// (0, pi/2) or (pi, 3pi/2) carry the sum: exp(tL) U = 2 Re sum_P c_j y_j.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <tuple>

#include "pa_engine.h"
#include "pa_rexi.h"

namespace pa {

using cplx = std::complex<double>;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Independent node indices of an N-node rule (N % 4 == 0).
std::vector<int> rexi_indep(int N) {
  std::vector<int> J;
  for (int j = 0; j < N / 4; j++) J.push_back(j);
  for (int j = N / 2; j < 3 * N / 4; j++) J.push_back(j);
  return J;
}

void rexi_node(int N, double eta0, int j, cplx &X, cplx &W) {
  const cplx w(eta0, 2.0 * kPi * (j + 0.5) / N);
  X = std::cosh(w);
  W = std::sinh(w) / (double)N;
}

// Largest |r(x) - exp(i theta x)| over 401 Chebyshev points of [-1, 1]
// (all N nodes summed), and the solve-error factor sum_j |c_j| / dist(X_j,
// [-1, 1]) of the rational sum.
void rexi_quality(double theta, int N, double eta0, double *err, double *amp) {
  std::vector<cplx> X(N), c(N);
  double a = 0.0;
  for (int j = 0; j < N; j++) {
    cplx W;
    rexi_node(N, eta0, j, X[j], W);
    c[j] = std::exp(cplx(0.0, theta) * X[j]) * W;
    // distance from X_j to the segment [-1, 1]
    const double xr = std::min(1.0, std::max(-1.0, X[j].real()));
    a += std::abs(c[j]) / std::abs(X[j] - xr);
  }
  double e = 0.0;
  for (int i = 0; i <= 400; i++) {
    const double x = std::cos(kPi * i / 400.0);
    cplx r = 0.0;
    for (int j = 0; j < N; j++) r += c[j] / (X[j] - x);
    e = std::max(e, std::abs(r - std::exp(cplx(0.0, theta * x))));
  }
  *err = e;
  *amp = a;
}

struct RexiChoice {
  int N = 0;
  double eta0 = 0.0;
};

// The pair (N, eta0) of smallest N / eta0 (iterations of a shifted solve
// grow like 1/eta0) with the rational function within tol/2 of the
// exponential at theta_max and the solve error factor times rtol below tol/2.
RexiChoice rexi_choose(double theta_max, double tol, double rtol) {
  static std::mutex mu;
  static std::map<std::tuple<double, double, double>, RexiChoice> cache;
  const auto key = std::make_tuple(theta_max, tol, rtol);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  RexiChoice best;
  double best_cost = 0.0;
  for (int k = 2; k <= 30; k++) {
    const double eta0 = 0.05 * k;
    auto ok = [&](int N) {
      double err, amp;
      rexi_quality(theta_max, N, eta0, &err, &amp);
      return err <= 0.5 * tol && amp * rtol <= 0.5 * tol;
    };
    if (!ok(256)) continue;
    int lo = 2, hi = 64;  // N = 4 lo fails (or is the smallest), N = 4 hi passes
    if (ok(8)) {
      hi = 2;
    } else {
      while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (ok(4 * mid)) hi = mid; else lo = mid;
      }
    }
    const int N = 4 * hi;
    const double cost = N / eta0;
    if (best.N == 0 || cost < best_cost) {
      best.N = N;
      best.eta0 = eta0;
      best_cost = cost;
    }
  }
  if (best.N == 0)
    throw Error(PA_EINVAL, "no rational approximation of at most 256 nodes meets cheb_tol at this "
                           "time span and cg_rtol");
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = best;
  return best;
}

int pad_to_tiles(int c) { return pad_cols(c); }
}  // namespace

// --------------------------------------------------------------- planning
void Engine::rexi_plan(RexiSys &rs, double theta_max, int members) {
  if (cfg_.rexi_nodes != 0) {
    if (cfg_.rexi_nodes % 4 != 0 || cfg_.rexi_nodes < 8 || cfg_.rexi_nodes > 256)
      throw Error(PA_EINVAL, "rexi_nodes must be a multiple of 4 in [8, 256]");
    if (!(cfg_.rexi_eta0 > 0.0 && cfg_.rexi_eta0 <= 3.0)) throw Error(PA_EINVAL, "rexi_eta0 in (0, 3]");
    rs.N = cfg_.rexi_nodes;
    rs.eta0 = cfg_.rexi_eta0;
  } else {
    const RexiChoice ch = rexi_choose(theta_max, cfg_.cheb_tol, cfg_.cg_rtol);
    rs.N = ch.N;
    rs.eta0 = ch.eta0;
  }
  rs.P = rs.N / 2;
  rs.members = members;
  rs.ncols = rs.P * members;
  rs.Bc = pad_to_tiles(rs.ncols);
  const double lb = ops_->lambda_bar, g = ops_->g, H = ops_->H;
  const std::vector<int> J = rexi_indep(rs.N);
  rs.X.resize(rs.P);
  rs.W.resize(rs.P);
  for (int jj = 0; jj < rs.P; jj++) rexi_node(rs.N, rs.eta0, J[jj], rs.X[jj], rs.W[jj]);
  // Schur coefficients per column: a = X, c = -gH/(lb^2 X), q = -i g/(lb X),
  // h = i H/(lb X), xinv = 1/X
  rs.hcoef.assign((size_t)5 * rs.Bc * 2, 0.0);
  const cplx I(0.0, 1.0);
  for (int col = 0; col < rs.ncols; col++) {
    const cplx X = rs.X[col % rs.P], xi = 1.0 / X;
    const cplx v[5] = {X, -g * H / (lb * lb) * xi, -I * (g / lb) * xi, I * (H / lb) * xi, xi};
    for (int f = 0; f < 5; f++) {
      rs.hcoef[2 * ((size_t)f * rs.Bc + col)] = v[f].real();
      rs.hcoef[2 * ((size_t)f * rs.Bc + col) + 1] = v[f].imag();
    }
  }
  const size_t bc = (size_t)rs.Bc;
  rs.coef = ar_.take<double2>(5 * bc);
  rs.rho = ar_.take<double2>(bc);
  rs.alpha = ar_.take<double2>(bc);
  rs.omega = ar_.take<double2>(bc);
  rs.beta = ar_.take<double2>(bc);
  rs.bb = ar_.take<double>(bc);
  rs.ff = ar_.take<double>(bc);
  rs.tau2 = ar_.take<double>(bc);
  rs.res2 = ar_.take<double>(bc);
  rs.active = ar_.take<int>(bc);
  rs.iters = ar_.take<int>(bc);
  rs.fresh = ar_.take<int>(bc);
  rs.restarts = ar_.take<int>(bc);
  rs.fail = ar_.take<int>(1);
  const size_t eb = (size_t)ne_ * bc;
  rs.Y = ar_.take<double2>((size_t)n_ * bc);
  rs.r = ar_.take<double2>(eb);
  rs.p[0] = ar_.take<double2>(eb);
  rs.p[1] = ar_.take<double2>(eb);
  rs.v[0] = ar_.take<double2>(eb);
  rs.v[1] = ar_.take<double2>(eb);
  rs.s = ar_.take<double2>(eb);
  rs.t = ar_.take<double2>(eb);
  // learned left preconditioner P / X (P the learned approximate inverse of
  // M_u bound to the operators) instead of Jacobi
  rs.learned = cfg_.precond == PA_PRECOND_LEARNED;
  if (rs.learned) {
    if (!ops_->lp_ready || !ops_->lp_dev)
      throw Error(PA_EINVAL, "no learned preconditioner bound to the operators");
    rs.w = ar_.take<double2>(eb);
  }
  rs.nwg = rexi_grid(ne_, rs.Bc);
  rs.part = ar_.take<double>((size_t)rs.nwg * 4 * bc);
}

// c_j(theta) of the P independent nodes, times `scale`.
void Engine::rexi_coefs(const RexiSys &rs, double theta, double scale, double2 *out) const {
  for (int jj = 0; jj < rs.P; jj++) {
    const cplx c = scale * std::exp(cplx(0.0, theta) * rs.X[jj]) * rs.W[jj];
    out[jj] = make_double2(c.real(), c.imag());
  }
}

void Engine::rexi_upload(RexiSys &rs) {
  upload(rs.coef, rs.hcoef.data(), rs.hcoef.size() * sizeof(double));
  stats.rexi_nodes = std::max(stats.rexi_nodes, rs.N);
  stats.rexi_eta0 = rs.eta0;
}

// ------------------------------------------------------------ the solves
// Solves every column's shifted system from the sources `src` into rs.Y
// (velocity rows by BiCGStab, depth rows from them).  Convergence is polled:
// first after the iteration count of the context's last solve, then every
// two iterations; a column whose preconditioned residual reached its target
// is checked against the true residual and restarted if it misses cg_rtol.
void Engine::rexi_solve(RexiSys &rs, const RexiSrc &src) {
  RexiArgs a{};
  a.ops = ops_->d;
  a.Bc = rs.Bc;
  a.P = rs.P;
  a.ncols = rs.ncols;
  a.binv = 1.0 / ops_->lambda_bar;
  a.co.a = rs.coef;
  a.co.c = rs.coef + rs.Bc;
  a.co.q = rs.coef + 2 * rs.Bc;
  a.co.h = rs.coef + 3 * rs.Bc;
  a.co.xinv = rs.coef + 4 * rs.Bc;
  a.src = src;
  a.x = rs.Y;  // velocity rows of the solution block
  a.r = rs.r;
  a.s = rs.s;
  a.t = rs.t;
  a.part = rs.part;
  a.max_wg = rs.nwg;
  a.st = RexiState{rs.rho, rs.alpha, rs.omega, rs.beta, rs.bb, rs.ff, rs.tau2, rs.res2,
                   rs.active, rs.iters, rs.fresh, rs.restarts, rs.fail};
  a.lp = rs.learned ? ops_->lp.p : nullptr;
  a.lpw = rs.learned ? ops_->lp.wp : 0;
  a.w = rs.w;
  a.seed = 0x5eed;
  a.rtol2 = cfg_.cg_rtol * cfg_.cg_rtol;
  a.maxit = cfg_.maxit;
  int par = 0;
  auto bind = [&] {
    a.p = rs.p[par];
    a.v = rs.v[par];
    a.p_next = rs.p[par ^ 1];
    a.v_next = rs.v[par ^ 1];
  };
  launch_zero((unsigned *)rs.fail, 1, s_);
  bind();
  a.mode = 0;
  launch_rexi_init(a, s_);
  if (a.lp) launch_rexi_lp(a, 0, s_);
  launch_rexi_fin_init(a, rs.nwg, s_);
  std::vector<int> act(rs.Bc);
  auto any_active = [&] {
    PA_HIP(hipMemcpyAsync(act.data(), rs.active, act.size() * sizeof(int), hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    for (int c = 0; c < rs.ncols; c++)
      if (act[c]) return true;
    return false;
  };
  int launched = 0;
  int chunk = ctx_ && ctx_->rexi_pred > 0 ? ctx_->rexi_pred : 8;
  bool more = true;
  while (more) {
    for (int k = 0; k < chunk && launched < cfg_.maxit; k++, launched++) {
      bind();
      launch_rexi_v(a, s_);
      if (a.lp) launch_rexi_lp(a, 1, s_);
      launch_rexi_fin_v(a, rs.nwg, s_);
      launch_rexi_t(a, s_);
      if (a.lp) launch_rexi_lp(a, 2, s_);
      launch_rexi_fin_t(a, rs.nwg, s_);
      launch_rexi_x(a, s_);
      launch_rexi_fin_x(a, rs.nwg, s_);
      par ^= 1;
    }
    if (any_active() && launched < cfg_.maxit) {
      chunk = 2;
      continue;
    }
    // true residual of every column; restarts for those that miss cg_rtol
    bind();
    a.mode = 1;
    launch_rexi_init(a, s_);
    if (a.lp) launch_rexi_lp(a, 0, s_);
    launch_rexi_fin_init(a, rs.nwg, s_);
    more = any_active() && launched < cfg_.maxit;
    chunk = 4;
  }
  // results of the solve
  std::vector<int> it(rs.Bc), rst(rs.Bc);
  std::vector<double> r2(rs.Bc), f2(rs.Bc);
  int fail = 0;
  PA_HIP(hipMemcpyAsync(it.data(), rs.iters, it.size() * sizeof(int), hipMemcpyDeviceToHost, s_));
  PA_HIP(hipMemcpyAsync(rst.data(), rs.restarts, rst.size() * sizeof(int), hipMemcpyDeviceToHost, s_));
  PA_HIP(hipMemcpyAsync(r2.data(), rs.res2, r2.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
  PA_HIP(hipMemcpyAsync(f2.data(), rs.ff, f2.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
  PA_HIP(hipMemcpyAsync(&fail, rs.fail, sizeof(int), hipMemcpyDeviceToHost, s_));
  sync_checked(s_);
  int imax = 0;
  for (int c = 0; c < rs.ncols; c++) {
    imax = std::max(imax, it[c]);
    stats.rexi_restarts += rst[c];
    if (f2[c] > 0) stats.rexi_resid_max = std::max(stats.rexi_resid_max, std::sqrt(r2[c] / f2[c]));
  }
  stats.rexi_solves++;
  if (rs.learned) {
    stats.precond = PA_PRECOND_LEARNED;
    stats.lp_solves++;
  }
  stats.rexi_iters += imax;
  stats.rexi_iters_max = std::max(stats.rexi_iters_max, imax);
  if (ctx_) ctx_->rexi_pred = std::max(2, imax);
  if (fail > 0 || any_active())
    throw Error(PA_ENOCONV, std::to_string(std::max(fail, 1)) +
                                " shifted solve column(s) did not reach cg_rtol within maxit");
  // depth rows
  RexiEtaArgs ea{};
  ea.ops = ops_->d;
  ea.Bc = rs.Bc;
  ea.P = rs.P;
  ea.ncols = rs.ncols;
  ea.co = a.co;
  ea.src = src;
  ea.yu = rs.Y;
  ea.yeta = rs.Y + (size_t)ne_ * rs.Bc;
  launch_rexi_eta(ea, s_);
}

// out[:, mem] = sum over the member's columns of Re(C[mem] Y) (expL: one
// coefficient row per member).
void Engine::rexi_combine(const RexiSys &rs, const double2 *C, int Go, int Mo, bool per_member,
                          double *out, int ostride) {
  RexiCombineArgs ca{};
  ca.n = n_;
  ca.Bc = rs.Bc;
  ca.P = rs.P;
  ca.members = rs.members;
  ca.Go = Go;
  ca.Mo = Mo;
  ca.per_member = per_member ? 1 : 0;
  ca.Y = rs.Y;
  ca.C = C;
  ca.out = out;
  ca.ostride = ostride;
  launch_rexi_combine(ca, s_);
}

// ------------------------------------------------------------ exponential
void Engine::rexi_exp_plan(RexiExp &x, RexiSys &rs, int B, const double *t) {
  x.B = B;
  x.Bs = pad_cols(B);
  x.hC.assign((size_t)B * rs.P, make_double2(0.0, 0.0));
  const double lb = ops_->lambda_bar;
  for (int b = 0; b < B; b++) rexi_coefs(rs, lb * t[b], 2.0, &x.hC[(size_t)b * rs.P]);
  x.C = ar_.take<double2>(std::max<size_t>(x.hC.size(), 1));
}

void Engine::rexi_exp_run(RexiExp &x, RexiSys &rs, Blk in, Blk out) {
  upload(x.C, x.hC.data(), x.hC.size() * sizeof(double2));
  RexiSrc src;
  src.real_blk = in.p;
  src.Bm = in.Bs;
  rexi_solve(rs, src);
  rexi_combine(rs, x.C, 1, 1, true, out.p, out.Bs);
}

void Engine::rexi_expL_apply(int B, const double *t, const double *Uin, double *Uout) {
  TuneScope tune_scope(tune_);
  double tmax = 0.0;
  for (int b = 0; b < B; b++) tmax = std::max(tmax, std::fabs(t[b]));
  const int Bs = pad_cols(B);
  plan_common(1);
  RexiSys rs;
  rexi_plan(rs, ops_->lambda_bar * tmax, B);
  RexiExp x;
  rexi_exp_plan(x, rs, B, t);
  Blk in = block(Bs), out = block(Bs);
  if (ar_.sizing()) return;
  begin();
  rexi_upload(rs);
  TransArgs tr{n_, B, Bs, const_cast<double *>(Uin), in.p};
  launch_to_block(tr, s_);
  rexi_exp_run(x, rs, in, out);
  TransArgs tb{n_, B, Bs, Uout, out.p};
  launch_from_block(tb, s_);
  finish();
}

// ------------------------------------------------------ averaged RHS
void Engine::rexi_nbar_plan(RexiNbar &nb, RexiSys &rs, const pa_avg *avg, int members) {
  const double lb = ops_->lambda_bar;
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
  const int P = rs.P, G = nb.G;
  nb.hCf.assign((size_t)G * P, make_double2(0.0, 0.0));
  nb.hCb.assign((size_t)nb.M * P, make_double2(0.0, 0.0));
  for (int i = 0; i < nb.M; i++) {
    const double s = avg->s[keep[i]], w = avg->w[keep[i]];
    rexi_coefs(rs, lb * s, 2.0, &nb.hCf[(size_t)i * P]);
    rexi_coefs(rs, -lb * s, w, &nb.hCb[(size_t)i * P]);
  }
  nb.hCs.assign((size_t)P, make_double2(2.0, 0.0));
  nb.hcolK.assign(nb.BsE, -1);
  for (int mem = 0; mem < members; mem++)
    for (int i = 0; i < nb.M; i++) nb.hcolK[mem * G + i] = 0;
  nb.Cf = ar_.take<double2>(nb.hCf.size());
  nb.Cb = ar_.take<double2>(nb.hCb.size());
  nb.Cs = ar_.take<double2>(nb.hCs.size());
  nb.colK = ar_.take<int>(nb.BsE);
  nb.E = ar_.take<double>((size_t)n_ * nb.BsE);
  nb.Yn = ar_.take<double>((size_t)n_ * nb.BsE);
  nb.Z = ar_.take<double2>((size_t)n_ * rs.Bc);
}

double Engine::rexi_theta_max(const pa_avg *avg) const {
  double smax = 0.0;
  for (double s : avg->s) smax = std::max(smax, std::fabs(s));
  return ops_->lambda_bar * smax;
}

void Engine::rexi_nbar_upload(RexiNbar &nb) {
  upload(nb.Cf, nb.hCf.data(), nb.hCf.size() * sizeof(double2));
  upload(nb.Cb, nb.hCb.data(), nb.hCb.size() * sizeof(double2));
  upload(nb.Cs, nb.hCs.data(), nb.hCs.size() * sizeof(double2));
  upload(nb.colK, nb.hcolK.data(), nb.hcolK.size() * sizeof(int));
}

// Nbar of the member block X into out (both [n][Bm]):
//   forward: P shared solves of X, E_m = 2 Re sum_j c_j(theta_m) y_j;
//   N of every E_m;
//   backward: Z_j = sum_m w_m c_j(-theta_m) N_m, P solves of Z_j,
//   Nbar = 2 Re sum_j y_j.
void Engine::rexi_nbar_run(RexiNbar &nb, RexiSys &rs, Blk X, Blk out) {
  RexiSrc fw;
  fw.real_blk = X.p;
  fw.Bm = X.Bs;
  rexi_solve(rs, fw);
  rexi_combine(rs, nb.Cf, nb.G, nb.M, false, nb.E, nb.BsE);
  nonlinear_block(Blk{nb.E, nb.BsE}, Blk{nb.Yn, nb.BsE}, nb.colK);
  RexiBackArgs ba{};
  ba.n = n_;
  ba.Bc = rs.Bc;
  ba.P = rs.P;
  ba.members = nb.members;
  ba.Gi = nb.G;
  ba.Mi = nb.M;
  ba.istride = nb.BsE;
  ba.Yn = nb.Yn;
  ba.C = nb.Cb;
  ba.Z = nb.Z;
  launch_rexi_back(ba, s_);
  RexiSrc bw;
  bw.cplx_blk = nb.Z;
  rexi_solve(rs, bw);
  rexi_combine(rs, nb.Cs, 1, 1, false, out.p, out.Bs);
  stats.terms += nb.M * nb.members;
}

void Engine::rexi_phase_avg_rhs(const pa_avg *avg, int members, const double *U, double *Nbar) {
  TuneScope tune_scope(tune_);
  if (members <= 0) throw Error(PA_EINVAL, "members must be positive");
  if (!(ops_->lambda_bar > 0)) throw Error(PA_EINVAL, "lambda_bar is not set");
  RexiSys rs;
  rexi_plan(rs, rexi_theta_max(avg), members);
  RexiNbar nb;
  rexi_nbar_plan(nb, rs, avg, members);
  plan_common(nb.BsE);
  C_ = ar_.take<double>((size_t)3 * nc_ * nb.BsE);
  Blk X = block(nb.Bm), out = block(nb.Bm);
  if (ar_.sizing()) return;
  begin();
  rexi_upload(rs);
  rexi_nbar_upload(nb);
  TransArgs tr{n_, members, nb.Bm, const_cast<double *>(U), X.p};
  launch_to_block(tr, s_);
  rexi_nbar_run(nb, rs, X, out);
  flush_check();
  TransArgs tb{n_, members, nb.Bm, Nbar, out.p};
  launch_from_block(tb, s_);
  finish();
}

// ---------------------------------------------------------------- RK4 step
// The stages of Engine::step with every exponential the rational sum (one
// node set for the averages and the stage exponentials, sized for the
// largest of T/2 and dt).
void Engine::rexi_step(const pa_avg *avg, double dt, int members, double *U) {
  TuneScope tune_scope(tune_);
  if (members <= 0) throw Error(PA_EINVAL, "members must be positive");
  if (!(ops_->lambda_bar > 0)) throw Error(PA_EINVAL, "lambda_bar is not set");
  RexiSys rs;
  rexi_plan(rs, std::max(rexi_theta_max(avg), ops_->lambda_bar * dt), members);
  RexiNbar nb;
  rexi_nbar_plan(nb, rs, avg, members);
  const int Bm = nb.Bm;
  plan_common(nb.BsE);
  C_ = ar_.take<double>((size_t)3 * nc_ * nb.BsE);
  std::vector<double> th(members, 0.5 * dt), tf(members, dt);
  RexiExp eh, ef;
  rexi_exp_plan(eh, rs, members, th.data());
  rexi_exp_plan(ef, rs, members, tf.data());
  Blk X = block(Bm), k1 = block(Bm), k2 = block(Bm), k3 = block(Bm), k4 = block(Bm);
  Blk Eh = block(Bm), T = block(Bm), S = block(Bm);
  if (ar_.sizing()) return;
  begin();
  rexi_upload(rs);
  rexi_nbar_upload(nb);
  const size_t nb_ = (size_t)n_ * Bm;
  TransArgs tr{n_, members, Bm, U, X.p};
  launch_to_block(tr, s_);
  rexi_nbar_run(nb, rs, X, k1);
  axpy(nb_, T.p, 1.0, X.p, 0.5 * dt, k1.p);  // U1
  rexi_exp_run(eh, rs, T, S);                 // exp(L dt/2) U1
  rexi_nbar_run(nb, rs, S, k2);
  rexi_exp_run(eh, rs, X, Eh);                // exp(L dt/2) U
  axpy(nb_, T.p, 1.0, Eh.p, 0.5 * dt, k2.p);  // U2
  rexi_nbar_run(nb, rs, T, k3);
  axpy(nb_, T.p, 1.0, Eh.p, dt, k3.p);        // U3
  rexi_exp_run(eh, rs, T, S);
  rexi_nbar_run(nb, rs, S, k4);
  axpy(nb_, T.p, 1.0, X.p, dt / 6.0, k1.p);
  rexi_exp_run(ef, rs, T, S);                 // exp(L dt)(U + dt/6 k1)
  axpy(nb_, T.p, dt / 3.0, k2.p, dt / 3.0, k3.p);
  rexi_exp_run(eh, rs, T, Eh);                // exp(L dt/2)(dt/3 (k2 + k3))
  axpy(nb_, X.p, 1.0, S.p, 1.0, Eh.p, dt / 6.0, k4.p);
  flush_check();
  TransArgs tb{n_, members, Bm, U, X.p};
  launch_from_block(tb, s_);
  finish();
}

}  // namespace pa
