// The paper's own pair of spaces (Sec. 2.5), BDM2 velocity x P1DG depth:
// host assembly of the linear operator of eq. ueq_int and the depth
// equation after it, and the Chebyshev exponential of Sec. 2.4 on it.
//
// Per flat triangle (its own plane, frame e1 = (p1 - p0)/|p1 - p0|,
// k = outward unit normal, e2 = k x e1): the velocity is any quadratic
// tangent field (12 coefficients), fixed by the normal component at the
// three Gauss-Legendre points of each edge (in the edge's global vertex
// order) and by the moments of u . e1 and u . e2 over |T| and of
// u . (x - x_T)^perp over |T|^1.5; the depth is linear (barycentric
// coefficients).  The local basis is the dual basis of those degrees of
// freedom, found by inverting their 12 x 12 matrix on scaled monomials
// about the centroid.  Integrals use the collapsed Gauss rule of 5 x 5
// points with barycentric points (1 - a - b(1 - a), a, b(1 - a)) in the
// cell's vertex order (exact to degree 8; the Coriolis parameter
// f = 2 Omega z/|x| is taken at its points).  Assembled:
//   M_u (ELL 21), F (same pattern), B (ELL 6), and per cell
//   Q = -H M_h^-1 B_T^T (the depth rows of L; M_h is block diagonal).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pa_bdm2.h"
#include "pa_engine.h"
#include "pa_kernels.h"

namespace pa {
namespace {

void bneed(bool ok, const char *msg) {
  if (!ok) throw Error(PA_EINVAL, msg);
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n).
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; i++) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; k++) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = (2/((1-z^2) P'^2)) / 2
  }
}

struct V2 {
  double x, y;
};

// Solve A X = I for a 12 x 12 matrix by Gauss-Jordan elimination with
// partial pivoting; A is destroyed.
void invert12(double A[12][12], double X[12][12]) {
  for (int i = 0; i < 12; i++)
    for (int j = 0; j < 12; j++) X[i][j] = i == j ? 1.0 : 0.0;
  for (int c = 0; c < 12; c++) {
    int p = c;
    for (int r = c + 1; r < 12; r++)
      if (std::fabs(A[r][c]) > std::fabs(A[p][c])) p = r;
    if (A[p][c] == 0.0) throw Error(PA_EINVAL, "BDM2 degrees of freedom are not unisolvent on a cell");
    for (int j = 0; j < 12; j++) {
      std::swap(A[c][j], A[p][j]);
      std::swap(X[c][j], X[p][j]);
    }
    const double inv = 1.0 / A[c][c];
    for (int j = 0; j < 12; j++) {
      A[c][j] *= inv;
      X[c][j] *= inv;
    }
    for (int r = 0; r < 12; r++) {
      if (r == c || A[r][c] == 0.0) continue;
      const double f = A[r][c];
      for (int j = 0; j < 12; j++) {
        A[r][j] -= f * A[c][j];
        X[r][j] -= f * X[c][j];
      }
    }
  }
}

// The 12 raw fields m_a(xi, eta) e_d, a < 6 over {1, xi, eta, xi^2, xi eta,
// eta^2} with (xi, eta) = (x - x_T)/h: values (2 components each) and
// divergences at a local point.
void raw_fields(V2 p, V2 cen, double h, double val[12][2], double div[12]) {
  const double xi = (p.x - cen.x) / h, et = (p.y - cen.y) / h;
  const double m[6] = {1.0, xi, et, xi * xi, xi * et, et * et};
  const double mx[6] = {0.0, 1.0, 0.0, 2.0 * xi, et, 0.0};  // d/dxi
  const double my[6] = {0.0, 0.0, 1.0, 0.0, xi, 2.0 * et};  // d/deta
  for (int a = 0; a < 6; a++) {
    val[2 * a][0] = m[a];
    val[2 * a][1] = 0.0;
    val[2 * a + 1][0] = 0.0;
    val[2 * a + 1][1] = m[a];
    div[2 * a] = mx[a] / h;
    div[2 * a + 1] = my[a] / h;
  }
}

// Add (col, m, f) to a velocity row of at most kB2W entries.
struct RowAcc {
  int n = 0;
  int col[kB2W];
  double m[kB2W], f[kB2W];
  void add(int c, double mv, double fv) {
    for (int i = 0; i < n; i++)
      if (col[i] == c) {
        m[i] += mv;
        f[i] += fv;
        return;
      }
    if (n == kB2W) throw Error(PA_EINVAL, "BDM2 row wider than 21");
    col[n] = c;
    m[n] = mv;
    f[n] = fv;
    n++;
  }
};
struct BRowAcc {
  int n = 0;
  int col[kB2WB];
  double v[kB2WB];
  void add(int c, double x) {
    for (int i = 0; i < n; i++)
      if (col[i] == c) {
        v[i] += x;
        return;
      }
    if (n == kB2WB) throw Error(PA_EINVAL, "BDM2 divergence row wider than 6");
    col[n] = c;
    v[n] = x;
    n++;
  }
};

}  // namespace

void bdm2_assemble(pa_bdm2 *b, const Mesh &m, const pa_phys &ph) {
  const int ne = m.ne(), nc = m.nc();
  b->ne = ne;
  b->nc = nc;
  b->nu = 3 * ne + 3 * nc;
  b->nh = 3 * nc;
  b->g = ph.g;
  b->H = ph.H;
  b->omega = ph.omega;
  b->lambda_bar = ph.lambda_bar;
  const int nu = b->nu;
  // collapsed Gauss rule (5 x 5) in barycentric coordinates
  std::vector<double> gx, gw;
  gauss_legendre01(5, gx, gw);
  std::vector<double> ql0, ql1, ql2, qw;
  for (int i = 0; i < 5; i++)
    for (int j = 0; j < 5; j++) {
      const double a = gx[i], bb = gx[j] * (1.0 - gx[i]);
      ql0.push_back(1.0 - a - bb);
      ql1.push_back(a);
      ql2.push_back(bb);
      qw.push_back(2.0 * gw[i] * gw[j] * (1.0 - gx[i]));  // sums to 1 over the triangle
    }
  const int nq = (int)qw.size();
  const double sq06 = std::sqrt(0.6);
  const double tg[3] = {0.5 - 0.5 * sq06, 0.5, 0.5 + 0.5 * sq06};

  std::vector<RowAcc> rows(nu);
  std::vector<BRowAcc> brows(nu);
  b->cdof.assign((size_t)12 * nc, 0);
  b->q.assign((size_t)36 * nc, 0.0);
  b->ncell.assign((size_t)kB2NC * nc, 0.0);
  b->mT.assign((size_t)144 * nc, 0.0);
  b->bot.assign((size_t)3 * nc, 0.0);
  b->rloc.assign((size_t)2 * nu, -1);
  b->etab.assign((size_t)4 * ne, -1);
  // volume and side rules of the nonlinear term
  b->qtab.resize(4 * (size_t)kB2VQ);
  for (int q = 0; q < kB2VQ; q++) {
    b->qtab[4 * q] = ql0[q];
    b->qtab[4 * q + 1] = ql1[q];
    b->qtab[4 * q + 2] = ql2[q];
    b->qtab[4 * q + 3] = qw[q];
  }
  {
    std::vector<double> fx, fw;
    gauss_legendre01(kB2FQ, fx, fw);
    b->ftab.resize(2 * (size_t)kB2FQ);
    for (int p = 0; p < kB2FQ; p++) {
      b->ftab[2 * p] = fx[p];
      b->ftab[2 * p + 1] = fw[p];
    }
  }
  for (int c = 0; c < nc; c++) {
    double P[3][3];
    for (int i = 0; i < 3; i++)
      for (int d = 0; d < 3; d++) P[i][d] = m.xyz[3 * m.tri[3 * c + i] + d];
    double u1[3], u2[3], k[3];
    for (int d = 0; d < 3; d++) {
      u1[d] = P[1][d] - P[0][d];
      u2[d] = P[2][d] - P[0][d];
    }
    k[0] = u1[1] * u2[2] - u1[2] * u2[1];
    k[1] = u1[2] * u2[0] - u1[0] * u2[2];
    k[2] = u1[0] * u2[1] - u1[1] * u2[0];
    const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    const double A = 0.5 * kn;
    const double l1 = std::sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    double e1[3], e2[3];
    for (int d = 0; d < 3; d++) {
      e1[d] = u1[d] / l1;
      k[d] /= kn;
    }
    e2[0] = k[1] * e1[2] - k[2] * e1[1];
    e2[1] = k[2] * e1[0] - k[0] * e1[2];
    e2[2] = k[0] * e1[1] - k[1] * e1[0];
    V2 x[3];
    for (int i = 0; i < 3; i++) {
      double dv[3];
      for (int d = 0; d < 3; d++) dv[d] = P[i][d] - P[0][d];
      x[i] = {dv[0] * e1[0] + dv[1] * e1[1] + dv[2] * e1[2], dv[0] * e2[0] + dv[1] * e2[1] + dv[2] * e2[2]};
    }
    const V2 cen = {(x[0].x + x[1].x + x[2].x) / 3.0, (x[0].y + x[1].y + x[2].y) / 3.0};
    const double h = std::sqrt(A);
    // degrees of freedom of the raw fields
    double Dm[12][12];
    int gid[12];
    double sg[12];
    V2 nside[3];
    for (int i = 0; i < 3; i++) {
      const int e = m.cedge[3 * c + i];
      const int va = m.evert[2 * e], vb = m.evert[2 * e + 1];
      int ia = -1, ib = -1;
      for (int v = 0; v < 3; v++) {
        if (m.tri[3 * c + v] == va) ia = v;
        if (m.tri[3 * c + v] == vb) ib = v;
      }
      bneed(ia >= 0 && ib >= 0 && ia != i && ib != i, "edge i of a cell must be opposite its vertex i");
      // outward unit normal of edge i in the plane
      const V2 pa_ = x[(i + 1) % 3], pb_ = x[(i + 2) % 3];
      V2 n = {pb_.y - pa_.y, -(pb_.x - pa_.x)};
      const V2 mid = {0.5 * (pa_.x + pb_.x), 0.5 * (pa_.y + pb_.y)};
      if (n.x * (mid.x - cen.x) + n.y * (mid.y - cen.y) < 0) {
        n.x = -n.x;
        n.y = -n.y;
      }
      const double nl = std::sqrt(n.x * n.x + n.y * n.y);
      n.x /= nl;
      n.y /= nl;
      nside[i] = n;
      const int sgn = (m.ecell[2 * e] == c) ? 1 : -1;
      b->etab[4 * e + (sgn > 0 ? 0 : 2)] = c;
      b->etab[4 * e + (sgn > 0 ? 1 : 3)] = i;
      for (int kq = 0; kq < 3; kq++) {
        const V2 p = {(1.0 - tg[kq]) * x[ia].x + tg[kq] * x[ib].x, (1.0 - tg[kq]) * x[ia].y + tg[kq] * x[ib].y};
        double val[12][2], dvv[12];
        raw_fields(p, cen, h, val, dvv);
        for (int f = 0; f < 12; f++) Dm[3 * i + kq][f] = val[f][0] * n.x + val[f][1] * n.y;
        gid[3 * i + kq] = 3 * e + kq;
        sg[3 * i + kq] = sgn;
      }
    }
    for (int mm = 0; mm < 3; mm++) {
      gid[9 + mm] = 3 * ne + 3 * c + mm;
      sg[9 + mm] = 1.0;
      for (int f = 0; f < 12; f++) Dm[9 + mm][f] = 0.0;
    }
    // quadrature points: local position, 3D position, weight
    std::vector<V2> qp(nq);
    std::vector<double> qf(nq), qa(nq);
    for (int q = 0; q < nq; q++) {
      const double b0 = ql0[q], b1 = ql1[q], b2 = ql2[q];
      qp[q] = {b0 * x[0].x + b1 * x[1].x + b2 * x[2].x, b0 * x[0].y + b1 * x[1].y + b2 * x[2].y};
      double X3[3];
      for (int d = 0; d < 3; d++) X3[d] = b0 * P[0][d] + b1 * P[1][d] + b2 * P[2][d];
      qf[q] = 2.0 * ph.omega * X3[2] / std::sqrt(X3[0] * X3[0] + X3[1] * X3[1] + X3[2] * X3[2]);
      qa[q] = qw[q] * A;
    }
    for (int q = 0; q < nq; q++) {
      double val[12][2], dvv[12];
      raw_fields(qp[q], cen, h, val, dvv);
      const V2 pp = {-(qp[q].y - cen.y), qp[q].x - cen.x};
      for (int f = 0; f < 12; f++) {
        Dm[9][f] += qa[q] * val[f][0] / A;
        Dm[10][f] += qa[q] * val[f][1] / A;
        Dm[11][f] += qa[q] * (val[f][0] * pp.x + val[f][1] * pp.y) / std::pow(A, 1.5);
      }
    }
    double C[12][12];
    invert12(Dm, C);  // column j of C: raw coefficients of basis function j
    {
      double *t = &b->ncell[(size_t)kB2NC * c];
      for (int f = 0; f < 12; f++)
        for (int j = 0; j < 12; j++) t[kNcC + 12 * f + j] = C[f][j];
      for (int r = 0; r < 3; r++) {
        t[kNcX + 2 * r] = (x[r].x - cen.x) / h;
        t[kNcX + 2 * r + 1] = (x[r].y - cen.y) / h;
        // grad l_r = k x (x_{r+2} - x_{r+1}) / 2A, k x (a, b) = (-b, a)
        const V2 d = {x[(r + 2) % 3].x - x[(r + 1) % 3].x, x[(r + 2) % 3].y - x[(r + 1) % 3].y};
        t[kNcGl + 2 * r] = -d.y / (2.0 * A);
        t[kNcGl + 2 * r + 1] = d.x / (2.0 * A);
        // side r: k x n_out = -n.y e1 + n.x e2 (3D), n_out, length, sign
        for (int dd = 0; dd < 3; dd++) t[kNcNp + 3 * r + dd] = -nside[r].y * e1[dd] + nside[r].x * e2[dd];
        t[kNcNo + 2 * r] = nside[r].x;
        t[kNcNo + 2 * r + 1] = nside[r].y;
        t[kNcLen + r] = std::sqrt(d.x * d.x + d.y * d.y);
        t[kNcSg + r] = sg[3 * r];
      }
      t[kNcH] = h;
      t[kNcA] = A;
      for (int dd = 0; dd < 3; dd++) {
        t[kNcE1 + dd] = e1[dd];
        t[kNcE2 + dd] = e2[dd];
      }
    }
    // element matrices
    double Ml[12][12] = {}, Fl[12][12] = {}, Bl[12][3] = {};
    for (int q = 0; q < nq; q++) {
      double val[12][2], dvv[12];
      raw_fields(qp[q], cen, h, val, dvv);
      double ph0[12], ph1[12], dph[12];
      for (int j = 0; j < 12; j++) {
        double s0 = 0, s1 = 0, sd = 0;
        for (int f = 0; f < 12; f++) {
          s0 += C[f][j] * val[f][0];
          s1 += C[f][j] * val[f][1];
          sd += C[f][j] * dvv[f];
        }
        ph0[j] = s0;
        ph1[j] = s1;
        dph[j] = sd;
      }
      const double lam[3] = {ql0[q], ql1[q], ql2[q]};
      for (int i = 0; i < 12; i++) {
        for (int j = 0; j < 12; j++) {
          Ml[i][j] += qa[q] * (ph0[i] * ph0[j] + ph1[i] * ph1[j]);
          // phi_i . (f k x phi_j), k x (a, b) = (-b, a) in the frame
          Fl[i][j] += qa[q] * qf[q] * (ph0[i] * -ph1[j] + ph1[i] * ph0[j]);
        }
        for (int r = 0; r < 3; r++) Bl[i][r] += qa[q] * dph[i] * lam[r];
      }
    }
    for (int i = 0; i < 12; i++) {
      for (int j = 0; j < 12; j++) {
        rows[gid[i]].add(gid[j], sg[i] * sg[j] * Ml[i][j], sg[i] * sg[j] * Fl[i][j]);
        b->mT[(size_t)144 * c + 12 * i + j] = sg[i] * sg[j] * Ml[i][j];
      }
      for (int r = 0; r < 3; r++) brows[gid[i]].add(3 * c + r, sg[i] * Bl[i][r]);
      b->cdof[12 * c + i] = gid[i];
      b->rloc[2 * (size_t)gid[i] + (b->rloc[2 * (size_t)gid[i]] < 0 ? 0 : 1)] = 12 * c + i;
    }
    // depth rows: -H M_h^-1 B_T^T, M_h^-1 = (12/A)(I - J/4)
    for (int qq = 0; qq < 3; qq++)
      for (int j = 0; j < 12; j++) {
        double s = 0.0;
        for (int r = 0; r < 3; r++) s += (12.0 / A) * ((qq == r ? 1.0 : 0.0) - 0.25) * sg[j] * Bl[j][r];
        b->q[((size_t)c * 3 + qq) * 12 + j] = -ph.H * s;
      }
  }
  // column-major ELL tables in block order: unknowns come in blocks of three
  // (an edge's points, a cell's moments) and the three rows of a block share
  // their columns, which are whole blocks (seven for an edge row: five edges
  // and two cells; four for a cell row, padded with the row's own block and
  // zero values).  Slot s = 3 b + k holds column 3 bid[b] + k, the block ids
  // ascending; one id table per row block serves its three rows.
  const int nb = nu / 3;
  b->bid.assign((size_t)kB2WBlk * nb, 0);
  b->col.assign((size_t)kB2W * nu, 0);
  b->mass.assign((size_t)kB2W * nu, 0.0);
  b->cor.assign((size_t)kB2W * nu, 0.0);
  b->bcol.assign((size_t)kB2WB * nu, 0);
  b->bval.assign((size_t)kB2WB * nu, 0.0);
  b->dinv.assign(nu, 0.0);
  for (int r = 0; r < nu; r++) {
    const RowAcc &ra = rows[r];
    int blk[kB2WBlk], nbk = 0;
    for (int s = 0; s < ra.n; s++) {
      const int bk = ra.col[s] / 3;
      bool seen = false;
      for (int t = 0; t < nbk; t++) seen |= blk[t] == bk;
      if (!seen) {
        if (nbk == kB2WBlk) throw Error(PA_EINVAL, "BDM2 row meets more than seven blocks");
        blk[nbk++] = bk;
      }
    }
    std::sort(blk, blk + nbk);
    if (3 * nbk != ra.n) throw Error(PA_EINVAL, "BDM2 row holds a partial block");
    for (int t = nbk; t < kB2WBlk; t++) blk[t] = r / 3;
    for (int t = 0; t < kB2WBlk; t++) {
      if (r % 3 == 0) b->bid[(size_t)t * nb + r / 3] = blk[t];
      else if (b->bid[(size_t)t * nb + r / 3] != blk[t])
        throw Error(PA_EINVAL, "rows of a BDM2 block differ in their columns");
      for (int k = 0; k < 3; k++) b->col[(size_t)(3 * t + k) * nu + r] = 3 * blk[t] + k;
    }
    for (int s = 0; s < ra.n; s++) {
      const int bk = ra.col[s] / 3, k = ra.col[s] % 3;
      int t = 0;
      while (blk[t] != bk) t++;
      b->mass[(size_t)(3 * t + k) * nu + r] = ra.m[s];
      b->cor[(size_t)(3 * t + k) * nu + r] = ra.f[s];
      if (ra.col[s] == r) b->dinv[r] = 1.0 / ra.m[s];
    }
    const BRowAcc &rb = brows[r];
    for (int s = 0; s < kB2WB; s++) {
      b->bcol[(size_t)s * nu + r] = s < rb.n ? rb.col[s] : 0;
      b->bval[(size_t)s * nu + r] = s < rb.n ? rb.v[s] : 0.0;
    }
  }
  // Ritz bounds of D^-1 M_u (as D^-1/2 M D^-1/2)
  std::vector<double> sq(nu);
  for (int i = 0; i < nu; i++) sq[i] = std::sqrt(b->dinv[i]);
  ritz_bounds(
      nu,
      [&](const std::vector<double> &v, std::vector<double> &w) {
        for (int i = 0; i < nu; i++) {
          double s = 0.0;
          for (int k2 = 0; k2 < kB2W; k2++) {
            const int cc = b->col[(size_t)k2 * nu + i];
            s += b->mass[(size_t)k2 * nu + i] * sq[cc] * v[cc];
          }
          w[i] = sq[i] * s;
        }
      },
      200, &b->eig_min, &b->eig_max);
}

// ------------------------------------------------------------- the calls
namespace {

enum { kCallL = PA_BDM2_APPLY_L, kCallExp = PA_BDM2_EXPL, kCallN = PA_BDM2_NONLINEAR, kCallNbar = PA_BDM2_PHASE_AVG };

// A call's plan: the mass solves' semi-iteration, the column passes
// (chunks of at most 64 columns) with their Chebyshev tables, and the
// workspace carve-up.
struct B2Plan {
  int call = 0, B = 0, Bs = 0, steps = 0, kmax = 0, nchunk = 1;
  double theta = 0.0;
  std::vector<double> c1, c2;
  std::vector<double> hF, hB;     // [nchunk][kmax + 1][Bs]: forward, backward weights
  std::vector<int32_t> cmem;      // [nchunk][Bs]: member of each column (-1: padding)
  std::vector<double> cw;         // [nchunk][Bs]: averaging weight of each column
  // shared-basis average (PA_BACKWARD_CLENSHAW): groups of G members
  bool shared = false;
  int G = 0, Gs = 0, Mk = 0, Vs = 0, nvch = 0, ngroup = 0;
  std::vector<double> cfh, cbh;   // [kmax + 1][Mk]: c_k(s_m), w_m c_k(-s_m)
  double *basis = nullptr, *Zs = nullptr, *V = nullptr, *Y = nullptr, *cfd = nullptr, *cbd = nullptr;
  double *eloc = nullptr;  // element-form step products [nc * 12][Bs] (wide blocks)
  // FP32 inner solves with FP64 refinement (PA_FP32_REFINED) on 64-column
  // blocks: rounds of kin steps, the last of klast, outer rounds in all
  bool mixed = false;
  int kin = 0, klast = 0, outer = 0;
  std::vector<double> mc1, mc2;
  float *r32 = nullptr, *y32[2] = {nullptr, nullptr};
  double *Ra = nullptr, *Rb = nullptr, *acc = nullptr, *r = nullptr, *dir[2] = {nullptr, nullptr};
  double *raw = nullptr, *ut = nullptr, *loc = nullptr, *rhs = nullptr;
  double *part = nullptr, *norms = nullptr, *coefF = nullptr, *coefB = nullptr, *cwd = nullptr;
  int32_t *cmemd = nullptr;
  int *fail = nullptr;
  unsigned long long *rmax = nullptr;
  // measurement hook (PA_KERNEL_B2_STEP): one event pair around the steps of
  // each mass solve, with the steps' algorithmic bytes and units
  pa_ctx *ctx = nullptr;
  mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> spans;
  mutable double prof_launches = 0, prof_bytes = 0, prof_units = 0;
};

hipEvent_t prof_event(pa_ctx *ctx) {
  if (!ctx->prof_pool.empty()) {
    hipEvent_t e = ctx->prof_pool.back();
    ctx->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PA_HIP(hipEventCreate(&e));
  return e;
}

// After the call's synchronisation: add the spans to the context's tally.
void prof_collect(const B2Plan &p) {
  if (!p.ctx || p.ctx->prof_kernel != PA_KERNEL_B2_STEP) return;
  for (auto &e : p.spans) {
    float t = 0;
    PA_HIP(hipEventElapsedTime(&t, e.first, e.second));
    p.ctx->prof_ms += t;
    p.ctx->prof_pool.push_back(e.first);
    p.ctx->prof_pool.push_back(e.second);
  }
  p.spans.clear();
  p.ctx->prof_launches += (int64_t)p.prof_launches;
  p.ctx->prof_work += (int64_t)p.prof_launches;
  p.ctx->prof_bytes += p.prof_bytes;
  p.ctx->prof_units += p.prof_units;
}

template <class T>
T *take(char *base, size_t &off, size_t cap, size_t n) {
  off = (off + 255) & ~(size_t)255;
  T *p = base ? (T *)(base + off) : nullptr;
  off += n * sizeof(T);
  if (base && off > cap) throw Error(PA_ENOMEM, "workspace too small");
  return p;
}

// Chebyshev weights of exp(t L) with lambda_bar lb: (2 - delta_k0) J_k(lb |t|)
// sign(t)^k, truncated at cheb_tol.
int exp_weights(double lb, double t, double tol, std::vector<double> &c) {
  const double theta = lb * std::fabs(t);
  if (!std::isfinite(theta) || theta > 1e7) throw Error(PA_EINVAL, "exponential time must be finite (lambda_bar |t| <= 1e7)");
  c = bessel_weights(theta, 2 * (int)std::ceil(theta) + 64);
  const int K = t == 0.0 ? 0 : truncate_degree(c, tol);
  c.resize(K + 1);
  if (t < 0)
    for (int k = 1; k <= K; k += 2) c[k] = -c[k];
  return K;
}

// Fill column chunk q's weights [kmax + 1][Bs] of the times tq (one per column).
void fill_weights(const pa_bdm2 *b, const std::vector<double> &tq, int Bs, int kmax, double tol,
                  double *dst) {
  std::vector<double> c;
  for (size_t j = 0; j < tq.size(); j++) {
    const int K = exp_weights(b->lambda_bar, tq[j], tol, c);
    for (int k = 0; k <= K && k <= kmax; k++) dst[(size_t)k * Bs + j] = c[k];
  }
}

size_t b2_plan(const pa_bdm2 *b, int call, int B, const double *t, const pa_avg *avg,
               const pa_solve_cfg &cfg, char *ws, size_t cap, B2Plan &p) {
  bneed(call >= kCallL && call <= kCallNbar, "unknown BDM2 call");
  p.call = call;
  p.B = B;
  const bool expo = call == kCallExp || call == kCallNbar;
  if (expo) bneed(b->lambda_bar > 0, "lambda_bar is not set");
  // Jacobi Chebyshev semi-iteration over the widened Ritz bounds
  const double lo = 0.97 * b->eig_min, hi = 1.01 * b->eig_max;
  if (!(lo > 0) || !(hi > lo)) throw Error(PA_EINVAL, "no spectral bounds of the BDM2 mass matrix");
  const double th = 0.5 * (lo + hi), de = 0.5 * (hi - lo), sigma = th / de;
  p.steps = std::min(cfg.maxit, (int)std::ceil(std::acosh(2.0 / cfg.cg_rtol) / std::acosh(sigma)) + 1);
  p.theta = th;
  p.c1.assign(p.steps, 0.0);
  p.c2.assign(p.steps, 0.0);
  double rho = 1.0 / sigma;
  for (int k = 0; k < p.steps; k++) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    p.c1[k] = rn * rho;
    p.c2[k] = 2.0 * rn / de;
    rho = rn;
  }
  p.mixed = cfg.precision == PA_FP32_REFINED;
  if (p.mixed) {
    // inner FP32 rounds to eps = max(inner_rtol, 1e-6) (the single-precision
    // floor), as many FP64 refinements as eps per round (counted as 10 eps)
    // needs to reach cg_rtol, the last round sized to the rest; the FP64
    // residual check of the solve decides
    const double eps = std::max(cfg.inner_rtol, 1e-6);
    p.kin = std::min(cfg.maxit, (int)std::ceil(std::acosh(2.0 / eps) / std::acosh(sigma)) + 1);
    p.outer = std::max(1, (int)std::ceil(std::log(cfg.cg_rtol) / std::log(10.0 * eps)));
    const double rest = cfg.cg_rtol / std::pow(eps, p.outer - 1);
    int kl = p.kin;
    if (rest > eps && rest < 1.0)
      kl = (int)std::ceil(std::acosh(2.0 / rest) / std::acosh(sigma)) + 1;
    else if (rest >= 1.0)
      kl = 1;
    p.klast = std::min(p.kin, std::max(kl, (p.kin + 1) / 2));
    p.mc1.assign(p.kin, 0.0);
    p.mc2.assign(p.kin, 0.0);
    double rh = 1.0 / sigma;
    for (int k = 0; k < p.kin; k++) {
      const double rn = 1.0 / (2.0 * sigma - rh);
      p.mc1[k] = rn * rh;
      p.mc2[k] = 2.0 * rn / de;
      rh = rn;
    }
  }
  std::vector<std::vector<double>> tF, tB;  // per chunk: forward and backward times
  p.shared = call == kCallNbar && cfg.backward == PA_BACKWARD_CLENSHAW;
  if (p.shared) {
    bneed(avg != nullptr, "no averaging nodes");
    double wmax = 0.0;
    for (double w : avg->w) wmax = std::max(wmax, w);
    std::vector<int> keep;
    for (size_t m = 0; m < avg->w.size(); m++)
      if (avg->w[m] >= cfg.weight_cut * wmax && avg->w[m] != 0.0) keep.push_back((int)m);
    bneed(!keep.empty(), "no averaging term left");
    p.Mk = (int)keep.size();
    std::vector<double> c;
    p.kmax = 0;
    for (int m : keep) p.kmax = std::max(p.kmax, exp_weights(b->lambda_bar, avg->s[m], cfg.cheb_tol, c));
    // up to 64 members share a basis (their node columns go through N 64 at
    // a time), fewer where the basis and the sums, 2 (kmax + 1) vectors a
    // member, would pass kB2BasisBytes
    const double per_col = 2.0 * (p.kmax + 1) * ((double)b->nu + b->nh) * sizeof(double);
    int gcap = 64;
    while (gcap > 1 && gcap * per_col > kB2BasisBytes) gcap /= 2;
    p.G = std::min(B, gcap);
    p.Gs = pad_cols(p.G);
    p.ngroup = (B + p.G - 1) / p.G;
    const int cols = p.G * p.Mk;
    p.Vs = pad_cols(std::min(cols, 64));
    p.nvch = (cols + p.Vs - 1) / p.Vs;
    p.Bs = p.Vs;  // the wide blocks (N and its solve)
    p.cfh.assign((size_t)(p.kmax + 1) * p.Mk, 0.0);
    p.cbh.assign((size_t)(p.kmax + 1) * p.Mk, 0.0);
    for (int i = 0; i < p.Mk; i++) {
      const int m = keep[i];
      int K = exp_weights(b->lambda_bar, avg->s[m], cfg.cheb_tol, c);
      for (int k = 0; k <= K; k++) p.cfh[(size_t)k * p.Mk + i] = c[k];
      K = exp_weights(b->lambda_bar, -avg->s[m], cfg.cheb_tol, c);
      for (int k = 0; k <= K; k++) p.cbh[(size_t)k * p.Mk + i] = avg->w[m] * c[k];
    }
    const size_t n = (size_t)b->nu + b->nh;
    size_t off = 0;
    p.basis = take<double>(ws, off, cap, (size_t)(p.kmax + 1) * n * p.Gs);
    p.Zs = take<double>(ws, off, cap, (size_t)(p.kmax + 1) * n * p.Gs);
    p.V = take<double>(ws, off, cap, n * p.Vs);
    p.Y = take<double>(ws, off, cap, n * p.Vs);
    p.r = take<double>(ws, off, cap, (size_t)b->nu * 64);
    p.dir[0] = take<double>(ws, off, cap, (size_t)b->nu * 64);
    p.dir[1] = take<double>(ws, off, cap, (size_t)b->nu * 64);
    p.raw = take<double>(ws, off, cap, (size_t)12 * b->nc * p.Vs);
    p.loc = take<double>(ws, off, cap, (size_t)12 * b->nc * p.Vs);
    p.ut = take<double>(ws, off, cap, (size_t)4 * kB2FQ * b->ne * p.Vs);
    p.rhs = take<double>(ws, off, cap, (size_t)b->nu * p.Vs);
    if (p.Vs >= kB2ElMin && p.Vs < 64) p.eloc = take<double>(ws, off, cap, (size_t)12 * b->nc * p.Vs);
    p.part = take<double>(ws, off, cap, (size_t)2048 * 64);
    if (p.mixed) {
      p.r32 = take<float>(ws, off, cap, (size_t)b->nu * 64);
      p.y32[0] = take<float>(ws, off, cap, (size_t)b->nu * 64);
      p.y32[1] = take<float>(ws, off, cap, (size_t)b->nu * 64);
    }
    p.norms = take<double>(ws, off, cap, (size_t)2 * 64);
    p.cfd = take<double>(ws, off, cap, p.cfh.size());
    p.cbd = take<double>(ws, off, cap, p.cbh.size());
    p.fail = take<int>(ws, off, cap, 2);
    p.rmax = take<unsigned long long>(ws, off, cap, 1);
    return off + 4096;
  }
  if (call == kCallNbar) {
    bneed(avg != nullptr, "no averaging nodes");
    double wmax = 0.0;
    for (double w : avg->w) wmax = std::max(wmax, w);
    std::vector<int> keep;
    for (size_t m = 0; m < avg->w.size(); m++)
      if (avg->w[m] >= cfg.weight_cut * wmax && avg->w[m] != 0.0) keep.push_back((int)m);
    const long cols = (long)B * (long)keep.size();
    bneed(cols > 0, "no averaging term left");
    p.Bs = pad_cols((int)std::min<long>(cols, 64));
    p.nchunk = (int)((cols + 63) / 64);
    p.cmem.assign((size_t)p.nchunk * p.Bs, -1);
    p.cw.assign((size_t)p.nchunk * p.Bs, 0.0);
    tF.resize(p.nchunk);
    tB.resize(p.nchunk);
    for (long c = 0; c < cols; c++) {
      const int q = (int)(c / 64), j = (int)(c % 64);
      const int mem = (int)(c / (long)keep.size()), m = keep[c % keep.size()];
      p.cmem[(size_t)q * p.Bs + j] = mem;
      p.cw[(size_t)q * p.Bs + j] = avg->w[m];
      tF[q].push_back(avg->s[m]);
      tB[q].push_back(-avg->s[m]);
    }
  } else {
    p.Bs = pad_cols(B);
    if (p.Bs > 64) throw Error(PA_ENOTSUP, "at most 64 states per BDM2 call");
    if (call == kCallExp) tF.assign(1, std::vector<double>(t, t + B));
  }
  p.kmax = 0;
  std::vector<double> c;
  for (auto &v : tF)
    for (double tj : v) p.kmax = std::max(p.kmax, exp_weights(b->lambda_bar, tj, cfg.cheb_tol, c));
  const size_t ctab = (size_t)(p.kmax + 1) * p.Bs;
  if (expo) {
    p.hF.assign(ctab * p.nchunk, 0.0);
    for (int q = 0; q < p.nchunk; q++) fill_weights(b, tF[q], p.Bs, p.kmax, cfg.cheb_tol, &p.hF[ctab * q]);
  }
  if (call == kCallNbar) {
    p.hB.assign(ctab * p.nchunk, 0.0);
    for (int q = 0; q < p.nchunk; q++) fill_weights(b, tB[q], p.Bs, p.kmax, cfg.cheb_tol, &p.hB[ctab * q]);
  }
  const int Bs = p.Bs;
  const size_t n = (size_t)b->nu + b->nh;
  size_t off = 0;
  p.Ra = take<double>(ws, off, cap, n * Bs);
  p.Rb = take<double>(ws, off, cap, n * Bs);
  if (expo) p.acc = take<double>(ws, off, cap, n * Bs);
  p.r = take<double>(ws, off, cap, (size_t)b->nu * Bs);
  p.dir[0] = take<double>(ws, off, cap, (size_t)b->nu * Bs);
  p.dir[1] = take<double>(ws, off, cap, (size_t)b->nu * Bs);
  if (call == kCallN || call == kCallNbar) {
    p.raw = take<double>(ws, off, cap, (size_t)12 * b->nc * Bs);
    p.loc = take<double>(ws, off, cap, (size_t)12 * b->nc * Bs);
    p.ut = take<double>(ws, off, cap, (size_t)4 * kB2FQ * b->ne * Bs);
    p.rhs = take<double>(ws, off, cap, (size_t)b->nu * Bs);
  }
  if (Bs >= kB2ElMin && Bs < 64) p.eloc = take<double>(ws, off, cap, (size_t)12 * b->nc * Bs);
  p.part = take<double>(ws, off, cap, (size_t)2048 * Bs);
  if (p.mixed && Bs == 64) {
    p.r32 = take<float>(ws, off, cap, (size_t)b->nu * 64);
    p.y32[0] = take<float>(ws, off, cap, (size_t)b->nu * 64);
    p.y32[1] = take<float>(ws, off, cap, (size_t)b->nu * 64);
  }
  p.norms = take<double>(ws, off, cap, (size_t)2 * Bs);
  if (expo) p.coefF = take<double>(ws, off, cap, p.hF.size());
  if (call == kCallNbar) {
    p.coefB = take<double>(ws, off, cap, p.hB.size());
    p.cmemd = take<int32_t>(ws, off, cap, p.cmem.size());
    p.cwd = take<double>(ws, off, cap, p.cw.size());
  }
  p.fail = take<int>(ws, off, cap, 2);
  p.rmax = take<unsigned long long>(ws, off, cap, 1);
  return off + 4096;
}

// The velocity solve M_u x = rhs (x starts at add_u) after k_b2_stiff set
// it up, then the residual check.
void b2_solve(const B2Plan &p, B2Args &a, hipStream_t s, pa_stats &st) {
  launch_b2_stiff(a, s);
  if (p.mixed && a.Bs == 64 && p.r32) {
    // FP32 inner rounds in the three-term form (the round's start y_1 from
    // k_b2_mix_init or the previous refinement, steps 2..kr over y_{k-1}),
    // each closed by an FP64 refinement of x and r; then the FP64 check of
    // |r|^2 against cg_rtol^2 |r_0|^2
    B2MixArgs m{};
    m.d = a.d;
    m.x = a.x;
    m.r = a.r;
    m.r32 = p.r32;
    m.part = a.part;
    m.theta_inv = (float)(1.0 / p.theta);
    float *cur = p.y32[0], *prev = p.y32[1];
    m.y_out = cur;
    launch_b2_mix_init(m, s);
    int steps = 0;
    for (int o = 0; o < p.outer; o++) {
      const int kr = o + 1 == p.outer ? p.klast : p.kin;
      steps += kr;
      for (int i = 1; i < kr; i++) {
        m.y_cur = cur;
        m.y_out = prev;
        m.c1 = (float)p.mc1[i - 1];
        m.c2 = (float)p.mc2[i - 1];
        m.zero_prev = i == 1 ? 1 : 0;
        launch_b2_cstep32(m, s);
        std::swap(cur, prev);
      }
      m.y_cur = cur;
      m.y_out = prev;
      m.last = o + 1 == p.outer ? 1 : 0;
      launch_b2_refine(m, s);
      std::swap(cur, prev);
    }
    launch_b2_check(a, s);
    st.solves++;
    st.refinements += p.outer;
    st.cg_iters += steps;
    st.cg_iters_max = std::max(st.cg_iters_max, steps);
    return;
  }
  const bool cel = a.Bs == 64;
  const bool el = !cel && a.Bs >= kB2ElMin && a.loc != nullptr;
  const bool prof = p.ctx && p.ctx->prof_kernel == PA_KERNEL_B2_STEP && p.steps > 0;
  if (prof) {
    p.spans.emplace_back(prof_event(p.ctx), prof_event(p.ctx));
    PA_HIP(hipEventRecord(p.spans.back().first, s));
    // per row and column four vectors (below); per row the ELL row (21
    // values, a third of seven block ids) and D^-1, or in the element and
    // cell forms per cell its 12 x 12 block and per row D^-1
    const double rows = a.d.nu, cols = a.Bs;
    const double mat = el || cel ? 1152.0 * a.d.nc + 8.0 * rows : (168.0 + 28.0 / 3.0 + 8.0) * rows;
    p.prof_launches += p.steps;
    // three-term: y_k, y_{k-1}, b in, y_{k+1} out; the finish x, y_K, b in, x out
    p.prof_bytes += p.steps * (mat + 32.0 * rows * cols);
    p.prof_units += (double)p.steps * cols;
  }
  // three-term form on the increment: y_1 = d_0 (set up in dir[0]), y_0 = 0
  // (step 1 does not read it); steps k = 1 .. K-1 write y_{k+1} over
  // y_{k-1}; the finish takes M y_K for the true residual (as many launches
  // as the two-term form, four vectors a step instead of six)
  for (int k = 1; k <= p.steps; k++) {
    a.dir_in = p.dir[(k + 1) & 1];   // y_k
    a.dir_out = p.dir[k & 1];        // y_{k-1} -> y_{k+1}
    a.first = k == 1;
    a.last = k == p.steps;
    if (!a.last) {
      a.c1 = p.c1[k - 1];
      a.c2 = p.c2[k - 1];
    }
    if (cel)
      launch_b2_cstep(a, s);
    else if (el)
      launch_b2_step3_el(a, s);
    else
      launch_b2_step3(a, s);
  }
  if (prof) PA_HIP(hipEventRecord(p.spans.back().second, s));
  launch_b2_check(a, s);
  st.solves++;
  st.cg_iters += p.steps;
  st.cg_iters_max = std::max(st.cg_iters_max, p.steps);
}

B2Args solve_args(const pa_bdm2 *b, const B2Plan &p, const pa_solve_cfg &cfg, int Bs) {
  B2Args a{};
  a.d = b->d;
  a.Bs = Bs;
  a.r = p.r;
  a.dir = p.dir[0];
  a.theta_inv = 1.0 / p.theta;
  a.part = p.part;
  a.norms = p.norms;
  a.rtol2 = cfg.cg_rtol * cfg.cg_rtol;
  a.fail = p.fail;
  a.rmax = p.rmax;
  a.loc = p.eloc;
  return a;
}

// out = scale L in + add (velocity: M_u^-1 (scale(-F u + g B eta)) + add_u
// as the solve from x_0 = add_u; depth: scale Q u + add_eta).
void b2_lapply(const pa_bdm2 *b, const B2Plan &p, const pa_solve_cfg &cfg, hipStream_t s, const double *in,
               double *out, const double *add, double scale, pa_stats &st, int Bs = 0) {
  if (Bs == 0) Bs = p.Bs;
  B2Args a = solve_args(b, p, cfg, Bs);
  const size_t nuB = (size_t)b->nu * Bs;
  a.scale = scale;
  a.u = in;
  a.eta = in + nuB;
  a.addu = add;
  a.adde = add ? add + nuB : nullptr;
  a.x = out;
  a.eta_out = out + nuB;
  b2_solve(p, a, s, st);
}

// out = N(in) (out must not alias in).
void b2_nl(const pa_bdm2 *b, const B2Plan &p, const pa_solve_cfg &cfg, hipStream_t s, const double *in,
           double *out, pa_stats &st) {
  const size_t nuB = (size_t)b->nu * p.Bs;
  B2NlArgs na{};
  na.d = b->d;
  na.Bs = p.Bs;
  na.u = in;
  na.eta = in + nuB;
  na.raw = p.raw;
  na.ut = p.ut;
  na.loc = p.loc;
  na.rhs = p.rhs;
  na.eta_out = out + nuB;
  launch_b2_nl(na, s);
  B2Args a = solve_args(b, p, cfg, p.Bs);
  a.scale = 1.0;
  a.u = in;
  a.eta = in + nuB;
  a.rhs = p.rhs;
  a.x = out;
  b2_solve(p, a, s, st);
}

// acc = sum_k c_k R_k with R_0 = Ra (overwritten), Rb scratch, coef the
// [kmax + 1][Bs] weights on the device.
void b2_exp(const pa_bdm2 *b, const B2Plan &p, const pa_solve_cfg &cfg, hipStream_t s, const double *coef,
            pa_stats &st) {
  const size_t nB = ((size_t)b->nu + b->nh) * p.Bs;
  AxpyArgs z{nB, 0.0, 0.0, 0.0, nullptr, nullptr, nullptr, p.acc};
  launch_axpy(z, s);
  auto accum = [&](const double *R, int k) {
    B2Args a{};
    a.d = b->d;
    a.Bs = p.Bs;
    a.u = R;
    a.eta = R + (size_t)b->nu * p.Bs;
    a.acc = p.acc;
    a.coef = coef + (size_t)k * p.Bs;
    launch_b2_acc(a, s);
  };
  accum(p.Ra, 0);
  double *prev = p.Ra, *cur = p.Rb;
  const double lb = b->lambda_bar;
  for (int k = 0; k < p.kmax; k++) {
    if (k == 0) {
      b2_lapply(b, p, cfg, s, prev, cur, nullptr, 1.0 / lb, st);
    } else {
      // R_{k+1} = (2/lb) L R_k + R_{k-1}, written over R_{k-1}
      b2_lapply(b, p, cfg, s, cur, prev, prev, 2.0 / lb, st);
      std::swap(prev, cur);
    }
    accum(cur, k + 1);
  }
  st.kmax = std::max(st.kmax, p.kmax);
}

template <class T>
void place(size_t &off, const std::vector<T> &v, const T **dst, char *base) {
  off = (off + 255) & ~(size_t)255;
  if (base) *dst = (const T *)(base + off);
  off += v.size() * sizeof(T);
}

size_t b2_layout(pa_bdm2 *b, char *base) {
  size_t off = 0;
  B2Dev d;
  place(off, b->bid, &d.bid, base);
  place(off, b->mass, &d.mass, base);
  place(off, b->cor, &d.cor, base);
  place(off, b->bcol, &d.bcol, base);
  place(off, b->bval, &d.bval, base);
  place(off, b->dinv, &d.dinv, base);
  place(off, b->cdof, &d.cdof, base);
  place(off, b->q, &d.q, base);
  place(off, b->ncell, &d.ncell, base);
  place(off, b->etab, &d.etab, base);
  place(off, b->rloc, &d.rloc, base);
  place(off, b->qtab, &d.qtab, base);
  place(off, b->ftab, &d.ftab, base);
  place(off, b->mT, &d.mT, base);
  place(off, b->mT32, &d.mT32, base);
  place(off, b->bot, &d.bot, base);
  if (base) {
    d.nu = b->nu;
    d.nh = b->nh;
    d.nc = b->nc;
    d.ne = b->ne;
    d.g = b->g;
    b->d = d;
  }
  return (off + 255) & ~(size_t)255;
}

template <class T>
void up(hipStream_t s, const T *dst, const std::vector<T> &v) {
  if (!v.empty())
    PA_HIP(hipMemcpyAsync((void *)dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// The pair's calls run FP64 Jacobi Chebyshev mass solves and the Chebyshev
// exponential only; settings asking for anything else are refused rather
// than ignored.
pa_solve_cfg cfg_of(const pa_solve_cfg *cfg) {
  pa_solve_cfg c;
  pa_solve_cfg_default(&c);
  if (cfg) c = *cfg;
  bneed(c.cg_rtol > 0 && c.cheb_tol > 0 && c.maxit > 0 && c.weight_cut >= 0, "bad solve configuration");
  bneed(c.backward == PA_BACKWARD_CLENSHAW || c.backward == PA_BACKWARD_PER_TERM, "unknown backward form");
  if (c.exponential != PA_EXP_CHEBYSHEV) throw Error(PA_ENOTSUP, "BDM2 calls take the Chebyshev exponential only");
  bneed(c.precision == PA_FP64 || c.precision == PA_FP32_REFINED, "unknown precision");
  if (c.solver != PA_SOLVER_CHEBYSHEV || c.precond != PA_PRECOND_JACOBI)
    throw Error(PA_ENOTSUP, "BDM2 mass solves are Jacobi Chebyshev semi-iterations only");
  return c;
}

// The call on a workspace: set-up, kernels, the solves' residual check.
void b2_run(pa_ctx *ctx, const pa_bdm2 *b, int call, int B, const double *t, const pa_avg *avg,
            const double *Uin, double *Uout, void *ws, size_t ws_bytes, const pa_solve_cfg &cfg,
            pa_stats *stats) {
  bneed(ctx && b && Uin && Uout && ws && B >= 1, "bad arguments");
  bneed(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  bneed(Uin != Uout, "outputs must not alias inputs");
  bneed(b->dev != nullptr, "BDM2 operators not bound (pa_bdm2_bind)");
  B2Plan p;
  b2_plan(b, call, B, t, avg, cfg, (char *)ws, ws_bytes, p);
  p.ctx = ctx;
  PA_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int n = b->nu + b->nh, Bs = p.Bs;
  pa_stats st{};
  hipEvent_t e0, e1;
  PA_HIP(hipEventCreate(&e0));
  PA_HIP(hipEventCreate(&e1));
  PA_HIP(hipEventRecord(e0, s));
  launch_zero((unsigned *)p.fail, 1, s);
  launch_zero((unsigned *)p.rmax, 2, s);
  if (p.coefF) PA_HIP(hipMemcpyAsync(p.coefF, p.hF.data(), p.hF.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (p.coefB) PA_HIP(hipMemcpyAsync(p.coefB, p.hB.data(), p.hB.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (p.cmemd) {
    PA_HIP(hipMemcpyAsync(p.cmemd, p.cmem.data(), p.cmem.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    PA_HIP(hipMemcpyAsync(p.cwd, p.cw.data(), p.cw.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if (p.shared) {
    // Nbar_j = sum_m w_m exp(-s_m L) N(exp(s_m L) U_j) with the exponentials
    // through each member's own basis: forward R_k = P_k(L) U_j on the
    // member's column (V(j, m) = sum_k c_k(s_m) R_k), N on the node columns,
    // backward Z_k = sum_m w_m c_k(-s_m) N(V(j, m)) summed by Clenshaw's
    // recurrence b_k = Z_k + (2/lb) L b_{k+1} + b_{k+2}, Nbar = Z_0 + b_2 +
    // (1/lb) L b_1 (P_1 = L / lb is half the general step).
    PA_HIP(hipMemcpyAsync(p.cfd, p.cfh.data(), p.cfh.size() * sizeof(double), hipMemcpyHostToDevice, s));
    PA_HIP(hipMemcpyAsync(p.cbd, p.cbh.data(), p.cbh.size() * sizeof(double), hipMemcpyHostToDevice, s));
    const size_t nG = (size_t)n * p.Gs;
    const double lb = b->lambda_bar;
    for (int g = 0; g < p.ngroup; g++) {
      const int j0 = g * p.G, gm = std::min(p.G, B - j0);
      TransArgs tr{n, gm, p.Gs, const_cast<double *>(Uin) + (size_t)j0 * n, p.basis};
      launch_to_block(tr, s);
      for (int k = 0; k < p.kmax; k++) {
        double *Rk = p.basis + k * nG, *Rn = p.basis + (k + 1) * nG;
        if (k == 0)
          b2_lapply(b, p, cfg, s, Rk, Rn, nullptr, 1.0 / lb, st, p.Gs);
        else
          b2_lapply(b, p, cfg, s, Rk, Rn, p.basis + (k - 1) * nG, 2.0 / lb, st, p.Gs);
      }
      AxpyArgs z0{nG * (p.kmax + 1), 0.0, 0.0, 0.0, nullptr, nullptr, nullptr, p.Zs};
      launch_axpy(z0, s);
      const int cols = gm * p.Mk;
      for (int col0 = 0; col0 < cols; col0 += p.Vs) {
        const int jlo = col0 / p.Mk, jhi = std::min(gm - 1, (col0 + p.Vs - 1) / p.Mk);
        B2BasisArgs ba{n,    p.Gs,  gm,      p.Mk,    p.Vs, col0, jlo, jhi - jlo + 1, p.kmax,
                       p.cfd, p.cbd, p.basis, p.V, p.Y, p.Zs};
        launch_b2_comb(ba, s);
        b2_nl(b, p, cfg, s, p.V, p.Y, st);
        launch_b2_zsum(ba, s);
      }
      for (int k = p.kmax - 1; k >= 0; k--) {
        double *Zk = p.Zs + k * nG;
        if (k + 2 <= p.kmax) {
          AxpyArgs ax{nG, 1.0, 1.0, 0.0, Zk, p.Zs + (k + 2) * nG, nullptr, Zk};
          launch_axpy(ax, s);
        }
        b2_lapply(b, p, cfg, s, p.Zs + (k + 1) * nG, Zk, Zk, (k == 0 ? 1.0 : 2.0) / lb, st, p.Gs);
      }
      TransArgs tb{n, gm, p.Gs, Uout + (size_t)j0 * n, p.Zs};
      launch_from_block(tb, s);
    }
    st.terms = B * p.Mk;
    st.kmax = p.kmax;
  } else if (call == kCallNbar) {
    // Nbar_j = sum_m w_m exp(-s_m L) N(exp(s_m L) U_j) over chunks of
    // (member, node) columns, accumulated in a fixed order
    launch_zero((unsigned *)Uout, (size_t)2 * n * B, s);
    const size_t ctab = (size_t)(p.kmax + 1) * Bs;
    for (int q = 0; q < p.nchunk; q++) {
      int jlo = B, jhi = -1;
      for (int c = 0; c < Bs; c++) {
        const int m = p.cmem[(size_t)q * Bs + c];
        if (m >= 0) {
          jlo = std::min(jlo, m);
          jhi = std::max(jhi, m);
        }
      }
      B2ColArgs ca{n, Bs, jlo, jhi - jlo + 1, p.cmemd + (size_t)q * Bs, p.cwd + (size_t)q * Bs, Uin, Uout,
                   p.Ra, p.acc};
      launch_b2_bcast(ca, s);
      b2_exp(b, p, cfg, s, p.coefF + ctab * q, st);
      b2_nl(b, p, cfg, s, p.acc, p.Ra, st);
      b2_exp(b, p, cfg, s, p.coefB + ctab * q, st);
      launch_b2_wsum(ca, s);
    }
    long cols = 0;
    for (int32_t m : p.cmem) cols += m >= 0;
    st.terms = (int32_t)cols;
  } else {
    TransArgs tr{n, B, Bs, const_cast<double *>(Uin), p.Ra};
    launch_to_block(tr, s);
    double *out_blk = p.Rb;
    if (call == kCallL) {
      b2_lapply(b, p, cfg, s, p.Ra, p.Rb, nullptr, 1.0, st);
    } else if (call == kCallN) {
      b2_nl(b, p, cfg, s, p.Ra, p.Rb, st);
    } else {
      b2_exp(b, p, cfg, s, p.coefF, st);
      out_blk = p.acc;
    }
    TransArgs tb{n, B, Bs, Uout, out_blk};
    launch_from_block(tb, s);
  }
  PA_HIP(hipEventRecord(e1, s));
  int fail = 0;
  unsigned long long rmax = 0;
  PA_HIP(hipMemcpyAsync(&fail, p.fail, sizeof(int), hipMemcpyDeviceToHost, s));
  PA_HIP(hipMemcpyAsync(&rmax, p.rmax, sizeof(rmax), hipMemcpyDeviceToHost, s));
  sync_checked(s);
  prof_collect(p);
  float ms = 0;
  PA_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st.device_ms = ms;
  std::memcpy(&st.resid_max, &rmax, sizeof(double));
  if (stats) *stats = st;
  if (fail > 0) throw Error(PA_ENOCONV, "a BDM2 mass solve missed cg_rtol");
}

// One step of the averaged system (Sec. 2.3), the Lawson RK4 form with
// exp(L dt/2) applied before the averages in stages 2 and 4 (it commutes
// with exp(L s)) and the last combination regrouped by linearity:
//   k1 = Nbar(U), k2 = Nbar(E (U + h k1)), k3 = Nbar(E U + h k2),
//   k4 = Nbar(E (E U + dt k3)),
//   U' = E (E (U + dt/6 k1) + dt/3 (k2 + k3)) + dt/6 k4,   E = exp(L h), h = dt/2.
// Member-major states; seven state buffers then the sub-calls' workspace.
size_t b2_step_ws(const pa_bdm2 *b, const pa_avg *avg, double dt, int B, const pa_solve_cfg &cfg,
                  char *ws, size_t cap, double **bufs) {
  bneed(B >= 1 && B <= 64, "at most 64 members per BDM2 step");
  bneed(dt > 0 && std::isfinite(dt), "dt must be positive and finite");
  const size_t nB = ((size_t)b->nu + b->nh) * B;
  size_t off = 0;
  for (int i = 0; i < 7; i++) {
    double *p = take<double>(ws, off, cap, nB);
    if (bufs) bufs[i] = p;
  }
  off = (off + 255) & ~(size_t)255;
  const std::vector<double> th(B, 0.5 * dt);
  B2Plan p1, p2;
  const size_t a = b2_plan(b, kCallNbar, B, nullptr, avg, cfg, nullptr, 0, p1);
  const size_t e = b2_plan(b, kCallExp, B, th.data(), nullptr, cfg, nullptr, 0, p2);
  return off + std::max(a, e);
}

void b2_step(pa_ctx *ctx, const pa_bdm2 *b, const pa_avg *avg, double dt, int B, double *U, void *ws,
             size_t ws_bytes, const pa_solve_cfg &cfg, pa_stats *stats) {
  bneed(ctx && b && avg && U && ws, "bad arguments");
  bneed(((uintptr_t)ws & 255) == 0, "workspace must be 256-byte aligned");
  double *k[7];
  const size_t need = b2_step_ws(b, avg, dt, B, cfg, (char *)ws, ws_bytes, k);
  bneed(need <= ws_bytes, "workspace too small");
  double *k1 = k[0], *k2 = k[1], *k3 = k[2], *k4 = k[3], *A = k[4], *Eh = k[5], *T = k[6];
  const size_t nB = ((size_t)b->nu + b->nh) * B;
  size_t sub_off = (7 * ((nB * sizeof(double) + 255) & ~(size_t)255) + 255) & ~(size_t)255;
  char *sub = (char *)ws + sub_off;
  const size_t sub_bytes = ws_bytes - sub_off;
  const std::vector<double> th(B, 0.5 * dt);
  const double h = 0.5 * dt;
  hipStream_t s = ctx->stream;
  pa_stats tot{};
  auto add = [&](const pa_stats &x) {
    tot.solves += x.solves;
    tot.cg_iters += x.cg_iters;
    tot.cg_iters_max = std::max(tot.cg_iters_max, x.cg_iters_max);
    tot.refinements += x.refinements;
    tot.kmax = std::max(tot.kmax, x.kmax);
    tot.terms += x.terms;
    tot.resid_max = std::max(tot.resid_max, x.resid_max);
    tot.device_ms += x.device_ms;
  };
  auto nbar = [&](const double *in, double *out) {
    pa_stats x{};
    b2_run(ctx, b, kCallNbar, B, nullptr, avg, in, out, sub, sub_bytes, cfg, &x);
    add(x);
  };
  auto expo = [&](const double *in, double *out) {
    pa_stats x{};
    b2_run(ctx, b, kCallExp, B, th.data(), nullptr, in, out, sub, sub_bytes, cfg, &x);
    add(x);
  };
  auto axpy = [&](double a0, const double *x0, double a1, const double *x1, double a2, const double *x2,
                  double *out) {
    AxpyArgs ax{nB, a0, a1, a2, x0, x1, x2, out};
    launch_axpy(ax, s);
  };
  nbar(U, k1);
  axpy(1.0, U, h, k1, 0.0, nullptr, A);
  expo(U, Eh);
  expo(A, T);
  nbar(T, k2);
  axpy(1.0, Eh, h, k2, 0.0, nullptr, A);
  nbar(A, k3);
  axpy(1.0, Eh, dt, k3, 0.0, nullptr, A);
  expo(A, T);
  nbar(T, k4);
  axpy(1.0, U, dt / 6.0, k1, 0.0, nullptr, A);
  expo(A, T);
  axpy(1.0, T, dt / 3.0, k2, dt / 3.0, k3, A);
  expo(A, T);
  axpy(1.0, T, dt / 6.0, k4, 0.0, nullptr, U);
  sync_checked(s);
  if (stats) *stats = tot;
}

// Power iteration for rho(L): L is skew in the energy inner product W, so
// -L^2 is W-symmetric with eigenvalues rho_j^2; v <- -L^2 v / |.|_W and the
// Rayleigh quotient |L v|_W^2 of the normalised v rises to rho^2.
double b2_estimate_lambda(pa_ctx *ctx, pa_bdm2 *b, int iters, void *ws, size_t ws_bytes) {
  pa_solve_cfg cfg;
  pa_solve_cfg_default(&cfg);
  cfg.cg_rtol = 1e-12;
  B2Plan p;
  b2_plan(b, kCallL, 1, nullptr, nullptr, cfg, (char *)ws, ws_bytes, p);
  PA_HIP(hipSetDevice(ctx->device));
  hipStream_t s = ctx->stream;
  const int n = b->nu + b->nh;
  // start vector from a counter hash (SplitMix64 of the index), in [-1, 1)
  std::vector<double> h(n);
  for (int i = 0; i < n; i++) {
    uint64_t z = (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    h[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  launch_zero((unsigned *)p.fail, 1, s);
  PA_HIP(hipMemcpyAsync(p.Ra, h.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  pa_stats st{};
  auto wnorm2 = [&](const double *x) {
    B2Args a{};
    a.d = b->d;
    a.Bs = 1;
    a.u = x;
    a.eta = x + b->nu;
    a.part = p.part;
    a.norms = p.norms;
    launch_b2_wnorm(a, b->H, s);
    double v = 0.0;
    PA_HIP(hipMemcpyAsync(&v, p.norms, sizeof(double), hipMemcpyDeviceToHost, s));
    sync_checked(s);
    return v;
  };
  double rho2 = 0.0;
  for (int it = 0; it < iters; it++) {
    const double nv = std::sqrt(wnorm2(p.Ra));
    AxpyArgs sc{(size_t)n, 1.0 / nv, 0.0, 0.0, p.Ra, nullptr, nullptr, p.Ra};
    launch_axpy(sc, s);
    b2_lapply(b, p, cfg, s, p.Ra, p.Rb, nullptr, 1.0, st);   // Rb = L v
    rho2 = wnorm2(p.Rb);
    b2_lapply(b, p, cfg, s, p.Rb, p.Ra, nullptr, -1.0, st);  // Ra = -L L v
  }
  int fail = 0;
  PA_HIP(hipMemcpyAsync(&fail, p.fail, sizeof(int), hipMemcpyDeviceToHost, s));
  sync_checked(s);
  if (fail > 0) throw Error(PA_ENOCONV, "a BDM2 mass solve missed its tolerance");
  return std::sqrt(rho2);
}

}  // namespace
}  // namespace pa

extern "C" {

int pa_mesh_from_arrays(int nv, const double *verts, int nc, const int32_t *cell_verts, int ne,
                        const int32_t *cell_edges, const int32_t *edge_cells, const int32_t *edge_verts,
                        double radius, pa_mesh **out) {
  return pa::guard([&] {
    pa::bneed(out && verts && cell_verts && cell_edges && edge_cells && edge_verts && nv > 0 && nc > 0 &&
                      ne > 0,
                  "bad arguments");
    auto *m = new pa_mesh;
    try {
      pa::Mesh &M = m->m;
      M.level = -1;
      M.radius = radius;
      M.xyz.assign(verts, verts + 3 * (size_t)nv);
      M.tri.assign(cell_verts, cell_verts + 3 * (size_t)nc);
      M.cedge.assign(cell_edges, cell_edges + 3 * (size_t)nc);
      M.ecell.assign(edge_cells, edge_cells + 2 * (size_t)ne);
      M.evert.assign(edge_verts, edge_verts + 2 * (size_t)ne);
      M.csgn.assign(3 * (size_t)nc, 0);
      pa::bneed(2 * (size_t)ne == 3 * (size_t)nc, "a closed triangulation has 2 ne = 3 nc");
      for (int v = 0; v < 3 * nc; v++) pa::bneed(M.tri[v] >= 0 && M.tri[v] < nv, "cell vertex out of range");
      for (int e = 0; e < ne; e++)
        pa::bneed(M.ecell[2 * e] >= 0 && M.ecell[2 * e] < M.ecell[2 * e + 1] && M.ecell[2 * e + 1] < nc,
                  "edge cells must satisfy 0 <= c0 < c1 < nc");
      for (int c = 0; c < nc; c++) {
        const double *p0 = &M.xyz[3 * M.tri[3 * c]], *p1 = &M.xyz[3 * M.tri[3 * c + 1]],
                     *p2 = &M.xyz[3 * M.tri[3 * c + 2]];
        const double a[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const double b[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        const double k[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        pa::bneed(k[0] * p0[0] + k[1] * p0[1] + k[2] * p0[2] > 0, "cells must be counter-clockwise seen from outside");
        for (int i = 0; i < 3; i++) {
          const int e = M.cedge[3 * c + i];
          pa::bneed(e >= 0 && e < ne, "cell edge out of range");
          const int va = M.tri[3 * c + (i + 1) % 3], vb = M.tri[3 * c + (i + 2) % 3];
          const bool first = M.ecell[2 * e] == c;
          pa::bneed(first || M.ecell[2 * e + 1] == c, "edge and cell tables disagree");
          // the edge runs a -> b counter-clockwise about its first cell
          const bool fwd = M.evert[2 * e] == va && M.evert[2 * e + 1] == vb;
          const bool rev = M.evert[2 * e] == vb && M.evert[2 * e + 1] == va;
          pa::bneed(first ? fwd : rev, "edge i of a cell must join its other two vertices, counter-clockwise about c0");
          M.csgn[3 * c + i] = first ? 1 : -1;
        }
      }
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

int pa_bdm2_create(const pa_mesh *m, const pa_phys *ph, pa_bdm2 **out) {
  return pa::guard([&] {
    pa::bneed(m && ph && out, "NULL argument");
    pa::bneed(ph->g > 0 && ph->H > 0 && ph->lambda_bar >= 0, "g and H must be positive");
    pa::bneed(ph->b_cell == nullptr, "no bottom topography in the BDM2 operator");
    auto *b = new pa_bdm2;
    try {
      b->mesh = m;
      pa::bdm2_assemble(b, m->m, *ph);
      b->mT32.assign(b->mT.begin(), b->mT.end());
      b->dev_bytes = pa::b2_layout(b, nullptr);
    } catch (...) {
      delete b;
      throw;
    }
    *out = b;
  });
}

int pa_bdm2_info(const pa_bdm2 *b, int32_t *nu, int32_t *nh, double *eig_min, double *eig_max) {
  return pa::guard([&] {
    pa::bneed(b != nullptr, "NULL argument");
    if (nu) *nu = b->nu;
    if (nh) *nh = b->nh;
    if (eig_min) *eig_min = b->eig_min;
    if (eig_max) *eig_max = b->eig_max;
  });
}

int pa_bdm2_tables(const pa_bdm2 *b, int32_t *col, double *mass, double *cor, int32_t *bcol, double *bval,
                   int32_t *cdof, double *q) {
  return pa::guard([&] {
    pa::bneed(b != nullptr, "NULL argument");
    auto cp = [](auto *dst, const auto &v) {
      if (dst) std::copy(v.begin(), v.end(), dst);
    };
    cp(col, b->col);
    cp(mass, b->mass);
    cp(cor, b->cor);
    cp(bcol, b->bcol);
    cp(bval, b->bval);
    cp(cdof, b->cdof);
    cp(q, b->q);
  });
}

int pa_bdm2_device_size(const pa_bdm2 *b, size_t *bytes) {
  return pa::guard([&] {
    pa::bneed(b && bytes, "NULL argument");
    *bytes = b->dev_bytes;
  });
}

int pa_bdm2_bind(pa_ctx *ctx, pa_bdm2 *b, void *dev_buf) {
  return pa::guard([&] {
    pa::bneed(ctx && b && dev_buf, "NULL argument");
    pa::bneed(((uintptr_t)dev_buf & 255) == 0, "device buffer must be 256-byte aligned");
    PA_HIP(hipSetDevice(ctx->device));
    b->dev = dev_buf;
    pa::b2_layout(b, (char *)dev_buf);
    hipStream_t s = ctx->stream;
    pa::up(s, b->d.bid, b->bid);
    pa::up(s, b->d.mass, b->mass);
    pa::up(s, b->d.cor, b->cor);
    pa::up(s, b->d.bcol, b->bcol);
    pa::up(s, b->d.bval, b->bval);
    pa::up(s, b->d.dinv, b->dinv);
    pa::up(s, b->d.cdof, b->cdof);
    pa::up(s, b->d.q, b->q);
    pa::up(s, b->d.ncell, b->ncell);
    pa::up(s, b->d.etab, b->etab);
    pa::up(s, b->d.rloc, b->rloc);
    pa::up(s, b->d.qtab, b->qtab);
    pa::up(s, b->d.ftab, b->ftab);
    pa::up(s, b->d.mT, b->mT);
    pa::up(s, b->d.mT32, b->mT32);
    pa::up(s, b->d.bot, b->bot);
    pa::sync_checked(s);
  });
}

int pa_bdm2_set_bottom(pa_bdm2 *b, const double *bottom_host) {
  return pa::guard([&] {
    pa::bneed(b != nullptr, "NULL argument");
    pa::bneed(b->dev == nullptr, "set the bottom before pa_bdm2_bind");
    if (bottom_host)
      std::copy(bottom_host, bottom_host + b->nh, b->bot.begin());
    else
      std::fill(b->bot.begin(), b->bot.end(), 0.0);
  });
}

int pa_bdm2_set_lambda(pa_bdm2 *b, double lambda_bar) {
  return pa::guard([&] {
    pa::bneed(b && lambda_bar > 0, "bad arguments");
    b->lambda_bar = lambda_bar;
  });
}

int pa_bdm2_workspace_size(const pa_bdm2 *b, int call, int B, const double *t_host, const pa_avg *avg,
                           const pa_solve_cfg *cfg, size_t *bytes) {
  return pa::guard([&] {
    pa::bneed(b && bytes && B >= 1, "bad arguments");
    if (call == PA_BDM2_EXPL || call == PA_BDM2_STEP) pa::bneed(t_host != nullptr, "t_host is NULL");
    if (call == PA_BDM2_STEP) {
      pa::bneed(avg != nullptr, "avg is NULL");
      *bytes = pa::b2_step_ws(b, avg, *t_host, B, pa::cfg_of(cfg), nullptr, 0, nullptr);
      return;
    }
    pa::B2Plan p;
    *bytes = pa::b2_plan(b, call, B, t_host, avg, pa::cfg_of(cfg), nullptr, 0, p);
  });
}

int pa_bdm2_apply_L(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *U_dev, double *out_dev, void *ws,
                    size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats) {
  return pa::guard([&] {
    pa::b2_run(ctx, b, PA_BDM2_APPLY_L, B, nullptr, nullptr, U_dev, out_dev, ws, ws_bytes, pa::cfg_of(cfg),
               stats);
  });
}

int pa_bdm2_expL_apply(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *t_host, const double *U_in_dev,
                       double *U_out_dev, void *ws, size_t ws_bytes, const pa_solve_cfg *cfg,
                       pa_stats *stats) {
  return pa::guard([&] {
    pa::bneed(t_host != nullptr, "t_host is NULL");
    pa::b2_run(ctx, b, PA_BDM2_EXPL, B, t_host, nullptr, U_in_dev, U_out_dev, ws, ws_bytes, pa::cfg_of(cfg),
               stats);
  });
}

int pa_bdm2_nonlinear(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *U_dev, double *out_dev, void *ws,
                      size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats) {
  return pa::guard([&] {
    pa::b2_run(ctx, b, PA_BDM2_NONLINEAR, B, nullptr, nullptr, U_dev, out_dev, ws, ws_bytes,
               pa::cfg_of(cfg), stats);
  });
}

int pa_bdm2_phase_avg_rhs(pa_ctx *ctx, const pa_bdm2 *b, const pa_avg *avg, int members, const double *U_dev,
                          double *Nbar_dev, void *ws, size_t ws_bytes, const pa_solve_cfg *cfg,
                          pa_stats *stats) {
  return pa::guard([&] {
    pa::bneed(avg != nullptr, "avg is NULL");
    pa::b2_run(ctx, b, PA_BDM2_PHASE_AVG, members, nullptr, avg, U_dev, Nbar_dev, ws, ws_bytes,
               pa::cfg_of(cfg), stats);
  });
}

int pa_bdm2_step(pa_ctx *ctx, const pa_bdm2 *b, const pa_avg *avg, double dt, int members, double *U_dev,
                 void *ws, size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats) {
  return pa::guard([&] { pa::b2_step(ctx, b, avg, dt, members, U_dev, ws, ws_bytes, pa::cfg_of(cfg), stats); });
}

int pa_bdm2_estimate_lambda(pa_ctx *ctx, pa_bdm2 *b, int iters, double safety, void *ws, size_t ws_bytes,
                            double *lambda_bar) {
  return pa::guard([&] {
    pa::bneed(ctx && b && ws, "bad arguments");
    pa::bneed(b->dev != nullptr, "BDM2 operators not bound (pa_bdm2_bind)");
    pa::bneed(iters >= 1 && safety >= 1.0, "need iters >= 1 and safety >= 1");
    b->lambda_bar = safety * pa::b2_estimate_lambda(ctx, b, iters, ws, ws_bytes);
    if (lambda_bar) *lambda_bar = b->lambda_bar;
  });
}

int pa_bdm2_destroy(pa_bdm2 *b) {
  return pa::guard([&] { delete b; });
}

}  // extern "C"
