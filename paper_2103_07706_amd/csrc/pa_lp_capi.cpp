// C ABI of the learned mass-matrix preconditioner (declared in include/pa.h):
// network parameters, training on the GPU with the library's own forward and
// backward kernels, the loss-gradient and inference hooks, and attaching the
// preconditioner P = G G^T to an operator.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include "pa_engine.h"
#include "pa_lp.h"

namespace pa {
namespace {

void lneed(bool ok, const char *msg) {
  if (!ok) throw Error(PA_EINVAL, msg);
}

// Workspace carving and kernel sequences of the network over one or more
// operator graphs (sizing pass when the workspace base is null).
class LpRunner {
 public:
  LpRunner(pa_ctx *ctx, const std::vector<const pa_ops *> &ops, int P, int bf16, int steps, void *ws,
           size_t ws_bytes)
      : s_(ctx ? ctx->stream : nullptr), P_(P), bf16_(bf16 != 0), ar_(ws, ws_bytes) {
    lneed(!ops.empty(), "no operators");
    lneed(P >= 1 && P <= kLpProbeMax, "probes must be in [1, 16]");
    L_ = lp_layout();
    int ne = 0, nc = 0;
    for (auto o : ops) {
      ne = std::max(ne, o->ne);
      nc = std::max(nc, o->nc);
    }
    theta_ = ar_.take<float>(L_.total);
    grad_ = ar_.take<double>(L_.total);
    m_ = ar_.take<double>(L_.total);
    v_ = ar_.take<double>(L_.total);
    for (int l = 0; l <= kLpLayers; l++) {
      he_[l] = ar_.take<float>((size_t)ne * 32);
      hc_[l] = ar_.take<float>((size_t)nc * 32);
    }
    z_ = ar_.take<float>((size_t)4 * ne * 32);
    gam_ = ar_.take<double>(ne);
    gd_ = ar_.take<double>(ne);
    goff_ = ar_.take<double>((size_t)4 * ne);
    dhe_ = ar_.take<float>((size_t)ne * 32);
    dhc_ = ar_.take<float>((size_t)nc * 32);
    dz_ = ar_.take<float>((size_t)4 * ne * 32);
    dxe_ = ar_.take<float>((size_t)ne * 64);
    dxc_ = ar_.take<float>((size_t)nc * 64);
    dxp_ = ar_.take<float>((size_t)4 * ne * 96);
    ddiag_ = ar_.take<double>(ne);
    doff_ = ar_.take<double>((size_t)4 * ne);
    part_ = ar_.take<double>((size_t)lp_wgrad_groups(4 * ne) * (96 * 32 + 32));
    const size_t pv = (size_t)ne * P;
    for (double **b : {&Z_, &y_, &w_, &a_, &res_, &t_, &u_}) *b = ar_.take<double>(pv);
    zinv_ = ar_.take<double>((size_t)kLpProbeMax * (ops.size() + 1));
    lpart_ = ar_.take<double>(lp_probe_groups(ne, P));
    nslots_ = std::max(1, steps) * (int)ops.size();
    loss_ = ar_.take<double>(nslots_);
    for (auto o : ops) {
      hosts_.push_back(std::unique_ptr<LpGraphHost>(new LpGraphHost(ar_.sizing() ? LpGraphHost{} : lp_graph(o))));
      graphs_.push_back(place_graph(o));
    }
    // 1 / |z|^2 of Rademacher probes per graph (slots 0..n-1); slot n for
    // probes given by the caller
    zinv_host_.assign((size_t)kLpProbeMax * (ops.size() + 1), 0.0);
    for (size_t gi = 0; gi < ops.size(); gi++)
      for (int p = 0; p < kLpProbeMax; p++) zinv_host_[gi * kLpProbeMax + p] = 1.0 / ops[gi]->ne;
    if (!ar_.sizing())
      PA_HIP(hipMemcpyAsync(zinv_, zinv_host_.data(), sizeof(double) * zinv_host_.size(),
                            hipMemcpyHostToDevice, s_));
  }

  size_t used() const { return ar_.used(); }
  bool sizing() const { return ar_.sizing(); }
  int ngraphs() const { return (int)graphs_.size(); }

  void upload_theta(const std::vector<float> &th) {
    PA_HIP(hipMemcpyAsync(theta_, th.data(), th.size() * sizeof(float), hipMemcpyHostToDevice, s_));
  }
  std::vector<float> download_theta() {
    std::vector<float> th(L_.total);
    PA_HIP(hipMemcpyAsync(th.data(), theta_, th.size() * sizeof(float), hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    return th;
  }
  void zero_grad() { launch_zero((unsigned *)grad_, (size_t)L_.total * 2, s_); }
  void zero_adam() {
    launch_zero((unsigned *)m_, (size_t)L_.total * 2, s_);
    launch_zero((unsigned *)v_, (size_t)L_.total * 2, s_);
  }

  void forward(int gi) {
    const LpGraphDev &g = graphs_[gi];
    LpDenseArgs a{};
    a.g = g;
    auto dense = [&](int kind, int W, int b, const float *hA, const float *hB, float *Y) {
      a.N = lp_rows(g, kind);
      a.W = theta_ + W;
      a.b = theta_ + b;
      a.hA = hA;
      a.hB = hB;
      a.Y = Y;
      launch_lp_dense_fwd(kind, bf16_, a, s_);
    };
    dense(LP_ENC_E, L_.ee_W, L_.ee_b, nullptr, nullptr, he_[0]);
    dense(LP_ENC_C, L_.ce_W, L_.ce_b, nullptr, nullptr, hc_[0]);
    for (int l = 0; l < kLpLayers; l++) {
      dense(LP_CELL, L_.cl_W[l], L_.cl_b[l], hc_[l], he_[l], hc_[l + 1]);
      dense(LP_EDGE, L_.el_W[l], L_.el_b[l], he_[l], hc_[l + 1], he_[l + 1]);
    }
    dense(LP_PAIR, L_.p1_W, L_.p1_b, he_[kLpLayers], hc_[kLpLayers], z_);
    LpHeadArgs h = heads(gi);
    launch_lp_heads_fwd(h, s_);
  }

  // loss into slot; gradient added to grad_ (probes already in Z_, zinv_)
  void loss_grad(int gi, int slot) {
    const LpGraphDev &g = graphs_[gi];
    LpProbeArgs pr{};
    pr.g = g;
    pr.P = P_;
    pr.gd = gd_;
    pr.goff = goff_;
    pr.z = Z_;
    pr.zinv = zcur_;
    pr.part = lpart_;
    auto G = [&](const double *in, double *out, int tr, double *res) {
      pr.in = in;
      pr.out = out;
      pr.transpose = tr;
      pr.res = res;
      launch_lp_probe_G(pr, s_);
    };
    auto M = [&](const double *in, double *out) {
      pr.in = in;
      pr.out = out;
      pr.res = nullptr;
      launch_lp_probe_M(pr, s_);
    };
    G(Z_, y_, 0, nullptr);
    M(y_, w_);
    G(w_, a_, 1, res_);
    launch_lp_loss_reduce(lpart_, lp_probe_groups(g.ne, P_), loss_ + slot, s_);
    G(res_, t_, 0, nullptr);
    M(t_, u_);
    LpGhatGradArgs gg{};
    gg.g = g;
    gg.P = P_;
    gg.w = w_;
    gg.res = res_;
    gg.u = u_;
    gg.z = Z_;
    gg.zinv = zcur_;
    gg.ddiag = ddiag_;
    gg.doff = doff_;
    launch_lp_ghat_grad(gg, s_);
    // heads
    LpHeadArgs h = heads(gi);
    launch_lp_heads_bwd(h, s_);
    vgrad(he_[kLpLayers], ddiag_, g.ne, L_.hd_w);
    vgrad(z_, doff_, 4 * g.ne, L_.p2_w);
    // pair layer
    LpDenseArgs a{};
    a.g = g;
    a.part = part_;
    auto back = [&](int kind, int W, const float *hA, const float *hB, const float *Y, const float *dY,
                    float *dX) {
      a.N = lp_rows(g, kind);
      a.W = theta_ + W;
      a.hA = hA;
      a.hB = hB;
      a.Y = const_cast<float *>(Y);  // read only in the backward kernels
      a.dY = dY;
      a.dX = dX;
      if (dX) launch_lp_dense_bwd(kind, bf16_, a, s_);
      launch_lp_wgrad(kind, bf16_, a, s_);
      const int KR = lp_in_dim(kind);
      launch_lp_wreduce(part_, lp_wgrad_groups(a.N), KR * 32 + 32, grad_ + W, s_);
    };
    back(LP_PAIR, L_.p1_W, he_[kLpLayers], hc_[kLpLayers], z_, dz_, dxp_);
    LpScatterArgs sc{};
    sc.g = g;
    sc.dxp = dxp_;
    sc.dxe = dxe_;
    sc.dxc = dxc_;
    sc.dhe = dhe_;
    sc.dhc = dhc_;
    sc.mode = LP_SC_PAIR;
    launch_lp_scatter(sc, s_);
    for (int l = kLpLayers - 1; l >= 0; l--) {
      back(LP_EDGE, L_.el_W[l], he_[l], hc_[l + 1], he_[l + 1], dhe_, dxe_);
      sc.mode = LP_SC_CELLS_FROM_EDGES;
      launch_lp_scatter(sc, s_);
      back(LP_CELL, L_.cl_W[l], hc_[l], he_[l], hc_[l + 1], dhc_, dxc_);
      sc.mode = LP_SC_EDGES;
      launch_lp_scatter(sc, s_);
      sc.mode = LP_SC_CELLS_DIRECT;
      launch_lp_scatter(sc, s_);
    }
    back(LP_ENC_E, L_.ee_W, nullptr, nullptr, he_[0], dhe_, nullptr);
    back(LP_ENC_C, L_.ce_W, nullptr, nullptr, hc_[0], dhc_, nullptr);
  }

  void set_probes_host(const double *Zh, const double *zinv_h) {
    zcur_ = zinv_ + (size_t)kLpProbeMax * graphs_.size();
    PA_HIP(hipMemcpyAsync(Z_, Zh, sizeof(double) * (size_t)graphs_[0].ne * P_, hipMemcpyHostToDevice, s_));
    PA_HIP(hipMemcpyAsync(zcur_, zinv_h, sizeof(double) * P_, hipMemcpyHostToDevice, s_));
    sync_checked(s_);
  }
  void set_probes_random(int gi, uint64_t seed) {
    launch_lp_rademacher(Z_, graphs_[gi].ne, P_, seed, s_);
    zcur_ = zinv_ + (size_t)kLpProbeMax * gi;
  }

  void adam(int step, double lr) {
    LpAdamArgs a{};
    a.n = L_.total;
    a.theta = theta_;
    a.grad = grad_;
    a.m = m_;
    a.v = v_;
    a.lr = lr;
    a.b1 = 0.9;
    a.b2 = 0.999;
    a.eps = 1e-8;
    a.c1 = 1.0 - std::pow(a.b1, step);
    a.c2 = 1.0 - std::pow(a.b2, step);
    a.gscale = 1.0 / ngraphs();
    launch_lp_adam(a, s_);
  }

  std::vector<double> losses() {
    std::vector<double> h(nslots_);
    PA_HIP(hipMemcpyAsync(h.data(), loss_, sizeof(double) * nslots_, hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    return h;
  }
  std::vector<double> grad_host() {
    std::vector<double> h(L_.total);
    PA_HIP(hipMemcpyAsync(h.data(), grad_, sizeof(double) * L_.total, hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
    return h;
  }
  void ghat_host(std::vector<double> &gd, std::vector<double> &goff) {
    const int ne = graphs_[0].ne;
    gd.resize(ne);
    goff.resize(4 * (size_t)ne);
    PA_HIP(hipMemcpyAsync(gd.data(), gd_, sizeof(double) * ne, hipMemcpyDeviceToHost, s_));
    PA_HIP(hipMemcpyAsync(goff.data(), goff_, sizeof(double) * 4 * ne, hipMemcpyDeviceToHost, s_));
    sync_checked(s_);
  }
  void sync() { sync_checked(s_); }
  hipStream_t stream() const { return s_; }

 private:
  LpHeadArgs heads(int gi) {
    LpHeadArgs h{};
    h.g = graphs_[gi];
    h.he = he_[kLpLayers];
    h.z = z_;
    h.w_hd = theta_ + L_.hd_w;
    h.b_hd = theta_ + L_.hd_b;
    h.w_p2 = theta_ + L_.p2_w;
    h.b_p2 = theta_ + L_.p2_b;
    h.gam = gam_;
    h.gd = gd_;
    h.goff = goff_;
    h.ddiag = ddiag_;
    h.doff = doff_;
    h.dhe = dhe_;
    h.dz = dz_;
    return h;
  }
  void vgrad(const float *X, const double *s, int N, int off) {
    LpVgradArgs v{};
    v.N = N;
    v.X = X;
    v.s = s;
    v.part = part_;
    launch_lp_vgrad(v, s_);
    launch_lp_wreduce(part_, lp_wgrad_groups(N), 33, grad_ + off, s_);
  }
  template <class T>
  const T *put(const std::vector<T> &h, size_t n) {
    T *d = ar_.take<T>(n);
    if (!ar_.sizing() && n)
      PA_HIP(hipMemcpyAsync(d, h.data(), n * sizeof(T), hipMemcpyHostToDevice, s_));
    return d;
  }
  LpGraphDev place_graph(const pa_ops *o) {
    const LpGraphHost &h = *hosts_.back();
    const size_t ne = o->ne, nc = o->nc;
    LpGraphDev d;
    d.ne = o->ne;
    d.nc = o->nc;
    d.Fe = put(h.Fe, ne * kLpFPad);
    d.Fc = put(h.Fc, nc * kLpFPad);
    d.ce = put(h.ce, nc * 3);
    d.ec = put(h.ec, ne * 2);
    d.pj = put(h.pj, ne * 4);
    d.pc = put(h.pc, ne * 4);
    d.tpos = put(h.tpos, ne * 4);
    d.revc = put(h.revc, nc * 6);
    d.mhat = put(h.mhat, ne * 4);
    d.mcol = put(h.mcol, ne * 5);
    d.mval = put(h.mval, ne * 5);
    return d;
  }

  hipStream_t s_;
  int P_;
  bool bf16_;
  Arena ar_;
  LpLayout L_;
  float *theta_ = nullptr;
  double *grad_ = nullptr, *m_ = nullptr, *v_ = nullptr;
  float *he_[kLpLayers + 1] = {}, *hc_[kLpLayers + 1] = {}, *z_ = nullptr;
  double *gam_ = nullptr, *gd_ = nullptr, *goff_ = nullptr;
  float *dhe_ = nullptr, *dhc_ = nullptr, *dz_ = nullptr, *dxe_ = nullptr, *dxc_ = nullptr, *dxp_ = nullptr;
  double *ddiag_ = nullptr, *doff_ = nullptr, *part_ = nullptr;
  double *Z_ = nullptr, *y_ = nullptr, *w_ = nullptr, *a_ = nullptr, *res_ = nullptr, *t_ = nullptr,
         *u_ = nullptr, *zinv_ = nullptr, *zcur_ = nullptr, *lpart_ = nullptr, *loss_ = nullptr;
  int nslots_ = 1;
  std::vector<double> zinv_host_;
  std::vector<std::unique_ptr<LpGraphHost>> hosts_;
  std::vector<LpGraphDev> graphs_;
};

std::vector<const pa_ops *> op_list(const pa_ops *const *ops, int n) {
  lneed(ops && n >= 1, "need at least one operator");
  std::vector<const pa_ops *> v;
  for (int i = 0; i < n; i++) {
    lneed(ops[i] != nullptr, "NULL operator");
    v.push_back(ops[i]);
  }
  return v;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace pa

extern "C" {

int pa_lp_create(int layers, int width, uint64_t seed, pa_lp **out) {
  return pa::guard([&] {
    pa::lneed(out != nullptr, "out is NULL");
    if (layers != pa::kLpLayers || width != pa::kLpW)
      throw pa::Error(PA_ENOTSUP, "only 3 message-passing rounds of width 32 are built");
    auto *lp = new pa_lp;
    lp->theta = pa::lp_init_params(seed);
    *out = lp;
  });
}

int pa_lp_param_count(const pa_lp *lp, int *n) {
  return pa::guard([&] {
    pa::lneed(lp && n, "NULL argument");
    *n = (int)lp->theta.size();
  });
}

int pa_lp_get_params(const pa_lp *lp, float *out) {
  return pa::guard([&] {
    pa::lneed(lp && out, "NULL argument");
    std::memcpy(out, lp->theta.data(), lp->theta.size() * sizeof(float));
  });
}

int pa_lp_set_params(pa_lp *lp, const float *in) {
  return pa::guard([&] {
    pa::lneed(lp && in, "NULL argument");
    std::memcpy(lp->theta.data(), in, lp->theta.size() * sizeof(float));
  });
}

int pa_lp_save(const pa_lp *lp, const char *path) {
  return pa::guard([&] {
    pa::lneed(lp && path, "NULL argument");
    FILE *f = std::fopen(path, "wb");
    if (!f) throw pa::Error(PA_EINVAL, std::string("cannot write ") + path);
    const char magic[8] = {'P', 'A', 'L', 'P', '0', '0', '0', '1'};
    const int32_t n = (int32_t)lp->theta.size();
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 &&
              std::fwrite(lp->theta.data(), 4, n, f) == (size_t)n;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw pa::Error(PA_EINVAL, std::string("write failed: ") + path);
  });
}

int pa_lp_load(pa_lp *lp, const char *path) {
  return pa::guard([&] {
    pa::lneed(lp && path, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) throw pa::Error(PA_EINVAL, std::string("cannot read ") + path);
    char magic[8];
    int32_t n = 0;
    std::vector<float> th(lp->theta.size());
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "PALP0001", 8) == 0 &&
                    std::fread(&n, 4, 1, f) == 1 && n == (int32_t)th.size() &&
                    std::fread(th.data(), 4, n, f) == (size_t)n;
    std::fclose(f);
    if (!ok) throw pa::Error(PA_EINVAL, std::string("not a parameter file of this network: ") + path);
    lp->theta = th;
  });
}

int pa_lp_destroy(pa_lp *lp) {
  return pa::guard([&] { delete lp; });
}

int pa_lp_workspace_size(const pa_ops *const *ops, int n_ops, int probes, int steps, size_t *bytes) {
  return pa::guard([&] {
    pa::lneed(bytes != nullptr, "bytes is NULL");
    pa::LpRunner r(nullptr, pa::op_list(ops, n_ops), probes, 1, steps, nullptr, 0);
    *bytes = r.used() + 4096;
  });
}

int pa_lp_train(pa_ctx *ctx, pa_lp *lp, const pa_ops *const *ops, int n_ops, const pa_train_cfg *cfg,
                void *ws, size_t ws_bytes, pa_train_stats *stats) {
  return pa::guard([&] {
    pa::lneed(ctx && lp && cfg && ws, "NULL argument");
    pa::lneed(cfg->steps >= 1 && cfg->lr > 0, "need steps >= 1 and lr > 0");
    PA_HIP(hipSetDevice(ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    pa::LpRunner r(ctx, pa::op_list(ops, n_ops), cfg->probes, cfg->bf16, cfg->steps, ws, ws_bytes);
    r.upload_theta(lp->theta);
    r.zero_adam();
    const int ng = r.ngraphs();
    for (int step = 1; step <= cfg->steps; step++) {
      r.zero_grad();
      for (int gi = 0; gi < ng; gi++) {
        r.set_probes_random(gi, cfg->seed * 0x100000001B3ull + (uint64_t)step * 1315423911ull + gi);
        r.forward(gi);
        r.loss_grad(gi, (step - 1) * ng + gi);
      }
      r.adam(step, cfg->lr);
    }
    lp->theta = r.download_theta();
    const std::vector<double> L = r.losses();
    const auto t1 = std::chrono::steady_clock::now();
    if (stats) {
      double first = 0.0, last = 0.0;
      for (int gi = 0; gi < ng; gi++) {
        first += L[gi];
        last += L[(size_t)(cfg->steps - 1) * ng + gi];
      }
      stats->loss_first = first / (ng * cfg->probes);
      stats->loss_last = last / (ng * cfg->probes);
      stats->steps = cfg->steps;
      stats->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
  });
}

int pa_lp_loss_grad(pa_ctx *ctx, const pa_lp *lp, const pa_ops *ops, int n_probe, const double *probes_host,
                    int bf16, void *ws, size_t ws_bytes, double *loss, double *grad_host) {
  return pa::guard([&] {
    pa::lneed(ctx && lp && ops && probes_host && ws && loss && grad_host, "NULL argument");
    PA_HIP(hipSetDevice(ctx->device));
    const pa_ops *one[1] = {ops};
    pa::LpRunner r(ctx, pa::op_list(one, 1), n_probe, bf16, 1, ws, ws_bytes);
    std::vector<double> zinv(n_probe, 0.0);
    for (int p = 0; p < n_probe; p++) {
      double s = 0.0;
      for (int i = 0; i < ops->ne; i++) s += probes_host[(size_t)i * n_probe + p] * probes_host[(size_t)i * n_probe + p];
      pa::lneed(s > 0, "a probe vector is zero");
      zinv[p] = 1.0 / s;
    }
    r.upload_theta(lp->theta);
    r.set_probes_host(probes_host, zinv.data());
    r.zero_grad();
    r.forward(0);
    r.loss_grad(0, 0);
    *loss = r.losses()[0] / n_probe;
    const std::vector<double> g = r.grad_host();
    std::memcpy(grad_host, g.data(), g.size() * sizeof(double));
  });
}

int pa_lp_ghat(pa_ctx *ctx, const pa_lp *lp, const pa_ops *ops, int bf16, void *ws, size_t ws_bytes,
               double *gdiag_host, double *goff_host) {
  return pa::guard([&] {
    pa::lneed(ctx && lp && ops && ws && gdiag_host && goff_host, "NULL argument");
    PA_HIP(hipSetDevice(ctx->device));
    const pa_ops *one[1] = {ops};
    pa::LpRunner r(ctx, pa::op_list(one, 1), 1, bf16, 1, ws, ws_bytes);
    r.upload_theta(lp->theta);
    r.forward(0);
    std::vector<double> gd, goff;
    r.ghat_host(gd, goff);
    std::memcpy(gdiag_host, gd.data(), gd.size() * sizeof(double));
    std::memcpy(goff_host, goff.data(), goff.size() * sizeof(double));
  });
}

int pa_ops_lp_attach(pa_ctx *ctx, pa_ops *ops, const pa_lp *lp, int bf16, void *ws, size_t ws_bytes,
                     pa_lp_info *info) {
  return pa::guard([&] {
    pa::lneed(ctx && ops && lp && ws, "NULL argument");
    PA_HIP(hipSetDevice(ctx->device));
    const pa_ops *one[1] = {ops};
    std::vector<double> gd, goff;
    {
      pa::LpRunner r(ctx, pa::op_list(one, 1), 1, bf16, 1, ws, ws_bytes);
      r.upload_theta(lp->theta);
      r.forward(0);
      r.ghat_host(gd, goff);
    }
    pa::lp_build_preconditioner(ops, gd, goff);
    if (info) {
      info->eig_min = ops->lp_eig_min;
      info->eig_max = ops->lp_eig_max;
      info->jacobi_eig_min = ops->mass_eig_min;
      info->jacobi_eig_max = ops->mass_eig_max;
      info->width_p = ops->lp_wp;
      info->width_pm = ops->lp_wpm;
    }
  });
}

int pa_ops_lp_device_size(const pa_ops *ops, size_t *bytes) {
  return pa::guard([&] {
    pa::lneed(ops && bytes, "NULL argument");
    pa::lneed(ops->lp_ready, "no learned preconditioner attached (pa_ops_lp_attach)");
    const size_t n1 = (size_t)ops->lp_wp * ops->ne, n2 = (size_t)ops->lp_wpm * ops->ne;
    *bytes = pa::al256(n1 * 8) + pa::al256(n2 * 8);
  });
}

int pa_ops_lp_bind(pa_ctx *ctx, pa_ops *ops, void *dev_buf) {
  return pa::guard([&] {
    pa::lneed(ctx && ops && dev_buf, "NULL argument");
    pa::lneed(ops->lp_ready, "no learned preconditioner attached (pa_ops_lp_attach)");
    pa::lneed(((uintptr_t)dev_buf & 255) == 0, "device buffer must be 256-byte aligned");
    PA_HIP(hipSetDevice(ctx->device));
    const size_t n1 = (size_t)ops->lp_wp * ops->ne, n2 = (size_t)ops->lp_wpm * ops->ne;
    auto pack = [](const std::vector<int32_t> &c, const std::vector<float> &v) {
      std::vector<uint2> out(c.size());
      for (size_t i = 0; i < c.size(); i++) {
        uint32_t bits;
        std::memcpy(&bits, &v[i], 4);
        out[i] = make_uint2((uint32_t)c[i], bits);
      }
      return out;
    };
    const std::vector<uint2> hp = pack(ops->lp_pcol, ops->lp_pval), hpm = pack(ops->lp_pmcol, ops->lp_pmval);
    char *b = (char *)dev_buf;
    pa::DevLp d;
    d.wp = ops->lp_wp;
    d.wpm = ops->lp_wpm;
    d.p = (const uint2 *)b;
    d.pm = (const uint2 *)(b + pa::al256(n1 * 8));
    hipStream_t s = ctx->stream;
    PA_HIP(hipMemcpyAsync((void *)d.p, hp.data(), n1 * 8, hipMemcpyHostToDevice, s));
    PA_HIP(hipMemcpyAsync((void *)d.pm, hpm.data(), n2 * 8, hipMemcpyHostToDevice, s));
    pa::sync_checked(s);
    ops->lp = d;
    ops->lp_dev = dev_buf;
    ops->gen = pa::next_generation();
  });
}

}  // extern "C"
