// Host side of the learned mass-matrix preconditioner: parameter layout and
// initialisation, the graph tables of an operator (features, pairs,
// transposes), and P = G G^T, P M with their spectral bounds.
#include <algorithm>
#include <cmath>

#include "pa_lp.h"

namespace pa {

LpLayout lp_layout() {
  LpLayout L{};
  int off = 0;
  auto take = [&](int n) {
    const int o = off;
    off += n;
    return o;
  };
  L.ee_W = take(kLpFE * kLpW);
  L.ee_b = take(kLpW);
  L.ce_W = take(kLpFC * kLpW);
  L.ce_b = take(kLpW);
  for (int l = 0; l < kLpLayers; l++) {
    L.cl_W[l] = take(2 * kLpW * kLpW);
    L.cl_b[l] = take(kLpW);
    L.el_W[l] = take(2 * kLpW * kLpW);
    L.el_b[l] = take(kLpW);
  }
  L.hd_w = take(kLpW);
  L.hd_b = take(1);
  L.p1_W = take(3 * kLpW * kLpW);
  L.p1_b = take(kLpW);
  L.p2_w = take(kLpW);
  L.p2_b = take(1);
  L.total = off;
  return L;
}

// Glorot-uniform weights (2u - 1) sqrt(6 / (fan_in + fan_out)) with u from
// SplitMix64(seed) (53-bit mantissas), drawn over the weight matrices in
// storage order; zero biases and zero output weights of both heads; the
// diagonal head's bias log(e - 1) makes the initial Ghat the identity.
std::vector<float> lp_init_params(uint64_t seed) {
  const LpLayout L = lp_layout();
  std::vector<float> th(L.total, 0.0f);
  uint64_t x = seed;
  auto uni = [&]() {
    x += 0x9E3779B97F4A7C15ull;
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int fin, int fout) {
    const double lim = std::sqrt(6.0 / (fin + fout));
    for (int i = 0; i < fin * fout; i++) th[off + i] = (float)((2.0 * uni() - 1.0) * lim);
  };
  fill(L.ee_W, kLpFE, kLpW);
  fill(L.ce_W, kLpFC, kLpW);
  for (int l = 0; l < kLpLayers; l++) {
    fill(L.cl_W[l], 2 * kLpW, kLpW);
    fill(L.el_W[l], 2 * kLpW, kLpW);
  }
  fill(L.p1_W, 3 * kLpW, kLpW);
  th[L.hd_b] = (float)std::log(std::exp(1.0) - 1.0);
  return th;
}

namespace {
struct P3 {
  double x, y, z;
};
P3 sub(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
double dot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
double len(P3 a) { return std::sqrt(dot(a, a)); }
}  // namespace

LpGraphHost lp_graph(const pa_ops *o) {
  const Mesh &m = o->mesh->m;
  const int ne = o->ne, nc = o->nc;
  LpGraphHost g;
  g.ne = ne;
  g.nc = nc;
  auto X = [&](int v) { return P3{m.xyz[3 * v], m.xyz[3 * v + 1], m.xyz[3 * v + 2]}; };
  // cosine of the angle of cell c at its vertex v
  auto cos_at = [&](int c, int v) {
    int k = 0;
    while (m.tri[3 * c + k] != v) k++;
    const P3 a = X(v), b = X(m.tri[3 * c + (k + 1) % 3]), d = X(m.tri[3 * c + (k + 2) % 3]);
    const P3 u = sub(b, a), w = sub(d, a);
    return dot(u, w) / (len(u) * len(w));
  };
  std::vector<double> elen(ne);
  double lbar = 0.0, abar = 0.0;
  for (int e = 0; e < ne; e++) {
    elen[e] = len(sub(X(m.evert[2 * e]), X(m.evert[2 * e + 1])));
    lbar += elen[e];
  }
  lbar /= ne;
  for (int c = 0; c < nc; c++) abar += o->area[c];
  abar /= nc;
  auto diag = [&](int e) { return o->mass[5 * e]; };
  g.Fe.assign((size_t)ne * kLpFPad, 0.0f);
  for (int e = 0; e < ne; e++) {
    const int a = m.evert[2 * e], b = m.evert[2 * e + 1];
    double opp[2], ends[4];
    for (int s = 0; s < 2; s++) {
      const int c = m.ecell[2 * e + s];
      int other = -1;
      for (int k = 0; k < 3; k++)
        if (m.tri[3 * c + k] != a && m.tri[3 * c + k] != b) other = m.tri[3 * c + k];
      opp[s] = cos_at(c, other);
      ends[2 * s] = cos_at(c, a);
      ends[2 * s + 1] = cos_at(c, b);
    }
    const P3 pa_ = X(a), pb = X(b);
    const P3 mid{0.5 * (pa_.x + pb.x), 0.5 * (pa_.y + pb.y), 0.5 * (pa_.z + pb.z)};
    const double emean = (ends[0] + ends[1] + ends[2] + ends[3]) / 4.0;
    const double emax = std::max(std::max(ends[0], ends[1]), std::max(ends[2], ends[3]));
    const double emin = std::min(std::min(ends[0], ends[1]), std::min(ends[2], ends[3]));
    const double f[kLpFE] = {diag(e),
                             elen[e] / lbar,
                             (o->area[m.ecell[2 * e]] + o->area[m.ecell[2 * e + 1]]) / (2.0 * abar),
                             mid.z / len(mid),
                             0.5 * (opp[0] + opp[1]),
                             std::fabs(opp[0] - opp[1]),
                             emean,
                             emax - emin};
    for (int k = 0; k < kLpFE; k++) g.Fe[(size_t)e * kLpFPad + k] = (float)f[k];
  }
  g.Fc.assign((size_t)nc * kLpFPad, 0.0f);
  for (int c = 0; c < nc; c++) {
    double cs[3];
    P3 cen{0, 0, 0};
    for (int k = 0; k < 3; k++) {
      const int v = m.tri[3 * c + k];
      cs[k] = cos_at(c, v);
      const P3 p = X(v);
      cen = {cen.x + p.x / 3.0, cen.y + p.y / 3.0, cen.z + p.z / 3.0};
    }
    const double f[kLpFC] = {
        o->area[c] / abar, cen.z / len(cen),
        std::max(cs[0], std::max(cs[1], cs[2])) - std::min(cs[0], std::min(cs[1], cs[2])),
        (diag(m.cedge[3 * c]) + diag(m.cedge[3 * c + 1]) + diag(m.cedge[3 * c + 2])) / 3.0};
    for (int k = 0; k < kLpFC; k++) g.Fc[(size_t)c * kLpFPad + k] = (float)f[k];
  }
  g.ce = m.cedge;
  g.ec = m.ecell;
  // pairs p = 4 i + s: row i, column = ELL slot s + 1 (slots 1, 2 in c0; 3, 4 in c1)
  g.pj.resize(4 * (size_t)ne);
  g.pc.resize(4 * (size_t)ne);
  g.mhat.resize(4 * (size_t)ne);
  for (int i = 0; i < ne; i++)
    for (int s = 0; s < 4; s++) {
      const int j = o->ell_col[5 * i + 1 + s];
      g.pj[4 * i + s] = j;
      g.pc[4 * i + s] = m.ecell[2 * i + (s < 2 ? 0 : 1)];
      g.mhat[4 * i + s] = o->mass[5 * i + 1 + s] / std::sqrt(diag(i) * diag(j));
    }
  g.tpos.resize(4 * (size_t)ne);
  for (int i = 0; i < ne; i++)
    for (int s = 0; s < 4; s++) {
      const int j = g.pj[4 * i + s];
      int t = -1;
      for (int u = 0; u < 4; u++)
        if (g.pj[4 * j + u] == i) t = 4 * j + u;
      if (t < 0) throw Error(PA_EINVAL, "mass pattern is not symmetric");
      g.tpos[4 * i + s] = t;
    }
  g.revc.assign(6 * (size_t)nc, -1);
  std::vector<int> fillc(nc, 0);
  for (int p = 0; p < 4 * ne; p++) {
    const int c = g.pc[p];
    if (fillc[c] >= 6) throw Error(PA_EINVAL, "cell with more than six pairs");
    g.revc[6 * c + fillc[c]++] = p;
  }
  for (int c = 0; c < nc; c++)
    if (fillc[c] != 6) throw Error(PA_EINVAL, "cell without six edge pairs");
  g.mcol = o->ell_col;
  g.mval.resize(5 * (size_t)ne);
  for (int i = 0; i < ne; i++)
    for (int j = 0; j < 5; j++)
      g.mval[5 * i + j] = o->mass[5 * i + j] / std::sqrt(diag(i) * diag(o->ell_col[5 * i + j]));
  return g;
}

namespace {
// Sparse row accumulator for the small products below.
struct RowAcc {
  std::vector<int> col;
  std::vector<double> val;
  void add(int c, double v) {
    for (size_t k = 0; k < col.size(); k++)
      if (col[k] == c) {
        val[k] += v;
        return;
      }
    col.push_back(c);
    val.push_back(v);
  }
  void clear() {
    col.clear();
    val.clear();
  }
};

// rows of a sparse matrix as (col, value) lists
struct Csr {
  std::vector<std::vector<int>> col;
  std::vector<std::vector<double>> val;
};

void to_ell(const Csr &A, int n, int *w, std::vector<int32_t> &col, std::vector<float> &val) {
  int width = 0;
  for (int i = 0; i < n; i++) width = std::max(width, (int)A.col[i].size());
  *w = width;
  col.assign((size_t)width * n, 0);
  val.assign((size_t)width * n, 0.0f);
  for (int i = 0; i < n; i++)
    for (int k = 0; k < width; k++) {
      const bool in = k < (int)A.col[i].size();
      col[(size_t)k * n + i] = in ? A.col[i][k] : i;
      val[(size_t)k * n + i] = in ? (float)A.val[i][k] : 0.0f;
    }
}
}  // namespace

void lp_build_preconditioner(pa_ops *o, const std::vector<double> &gd, const std::vector<double> &goff) {
  const int ne = o->ne;
  const LpGraphHost g = lp_graph(o);
  std::vector<double> rs(ne);  // D^-1/2
  for (int i = 0; i < ne; i++) rs[i] = 1.0 / std::sqrt(o->mass[5 * i]);
  // G = D^-1/2 Ghat, row i: (i, gd_i rs_i), (pj[p], goff[p] rs_i)
  auto g_row = [&](int i, int *cols, double *vals) {
    cols[0] = i;
    vals[0] = gd[i] * rs[i];
    for (int s = 0; s < 4; s++) {
      cols[1 + s] = g.pj[4 * i + s];
      vals[1 + s] = goff[4 * i + s] * rs[i];
    }
  };
  // column k of G: (k, G_kk) and (j, G_jk) for the pairs (j, k) = tpos of (k, j)
  auto g_col = [&](int k, int *rows, double *vals) {
    rows[0] = k;
    vals[0] = gd[k] * rs[k];
    for (int s = 0; s < 4; s++) {
      const int j = g.pj[4 * k + s];
      rows[1 + s] = j;
      vals[1 + s] = goff[g.tpos[4 * k + s]] * rs[j];
    }
  };
  Csr P, PM;
  P.col.resize(ne);
  P.val.resize(ne);
  PM.col.resize(ne);
  PM.val.resize(ne);
  RowAcc acc;
  for (int i = 0; i < ne; i++) {  // P_ij = sum_k G_ik G_jk
    int ci[5], rk[5];
    double vi[5], vk[5];
    g_row(i, ci, vi);
    acc.clear();
    for (int a = 0; a < 5; a++) {
      g_col(ci[a], rk, vk);
      for (int b = 0; b < 5; b++) acc.add(rk[b], vi[a] * vk[b]);
    }
    P.col[i] = acc.col;
    P.val[i] = acc.val;
  }
  for (int i = 0; i < ne; i++) {  // (P M)_ij = sum_k P_ik M_kj
    acc.clear();
    for (size_t a = 0; a < P.col[i].size(); a++) {
      const int k = P.col[i][a];
      for (int b = 0; b < 5; b++) acc.add(o->ell_col[5 * k + b], P.val[i][a] * o->mass[5 * k + b]);
    }
    PM.col[i] = acc.col;
    PM.val[i] = acc.val;
  }
  to_ell(P, ne, &o->lp_wp, o->lp_pcol, o->lp_pval);
  to_ell(PM, ne, &o->lp_wpm, o->lp_pmcol, o->lp_pmval);
  // spectrum of P M = that of Ghat^T Mhat Ghat
  ritz_bounds(
      ne,
      [&](const std::vector<double> &v, std::vector<double> &w) {
        std::vector<double> y(ne), t(ne);
        for (int i = 0; i < ne; i++) {  // y = Ghat v
          double s = gd[i] * v[i];
          for (int u = 0; u < 4; u++) s += goff[4 * i + u] * v[g.pj[4 * i + u]];
          y[i] = s;
        }
        for (int i = 0; i < ne; i++) {  // t = Mhat y
          double s = 0.0;
          for (int j = 0; j < 5; j++) s += g.mval[5 * i + j] * y[g.mcol[5 * i + j]];
          t[i] = s;
        }
        for (int i = 0; i < ne; i++) {  // w = Ghat^T t
          double s = gd[i] * t[i];
          for (int u = 0; u < 4; u++) s += goff[g.tpos[4 * i + u]] * t[g.pj[4 * i + u]];
          w[i] = s;
        }
      },
      200, &o->lp_eig_min, &o->lp_eig_max);
  o->lp_ready = true;
  o->gen = next_generation();
  o->lp_dev = nullptr;  // tables changed: bind again
}

}  // namespace pa
