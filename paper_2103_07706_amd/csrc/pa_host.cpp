// Host side of libpa: icosahedral mesh, RT0/P0 operator assembly into ELL
// arrays and the geometry tables of the nonlinear kernels.
//
// Mesh: the paper's experiments run on icosahedral grids (Sec. 3).  Level 0
// is the icosahedron, each refinement quarters every triangle at its edge
// midpoints, which are projected radially onto the sphere.
//
// Operators (Sec. 2.5, discrete L): with the RT0 basis function of local
// edge i of a flat triangle T, phi_i = s_i (x - p_i) / (2|T|) (p_i the vertex
// opposite edge i, s_i = +1 when the edge normal points out of T),
//   M_ij = int_T phi_i . phi_j         (exact, from vertex values),
//   F_ij = int_T f phi_i . (k x phi_j) (edge-midpoint rule, f = 2 Omega sin lat),
//   D_Te = s_Te,   area_T = |T|.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <unordered_map>

#include "pa_internal.h"
#include "pa_kernels.h"

namespace pa {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

V3 vert(const Mesh &m, int v) { return {m.xyz[3 * v], m.xyz[3 * v + 1], m.xyz[3 * v + 2]}; }

}  // namespace

Mesh build_icosahedral(int level, double radius) {
  if (level < 0 || level > 9) throw Error(PA_EINVAL, "mesh level must be in [0, 9]");
  if (!(radius > 0)) throw Error(PA_EINVAL, "radius must be positive");
  Mesh m;
  m.level = level;
  m.radius = radius;
  const double t = 0.5 * (1.0 + std::sqrt(5.0));
  // icosahedron: cyclic permutations of (0, +-1, +-t)
  std::vector<V3> P;
  for (int a = -1; a <= 1; a += 2)
    for (int b = -1; b <= 1; b += 2) {
      P.push_back({0.0, (double)a, b * t});
      P.push_back({(double)a, b * t, 0.0});
      P.push_back({b * t, 0.0, (double)a});
    }
  // faces: vertex triples whose three sides all have the minimal length 2
  std::vector<int32_t> T;
  for (int i = 0; i < 12; i++)
    for (int j = i + 1; j < 12; j++) {
      if (std::fabs(norm(P[i] - P[j]) - 2.0) > 1e-9) continue;
      for (int k = j + 1; k < 12; k++)
        if (std::fabs(norm(P[i] - P[k]) - 2.0) < 1e-9 &&
            std::fabs(norm(P[j] - P[k]) - 2.0) < 1e-9) {
          T.push_back(i);
          T.push_back(j);
          T.push_back(k);
        }
    }
  for (auto &p : P) p = (radius / norm(p)) * p;

  for (int l = 0; l < level; l++) {
    std::unordered_map<uint64_t, int32_t> mid;
    mid.reserve(T.size());
    auto midpoint = [&](int32_t a, int32_t b) {
      uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
      auto it = mid.find(key);
      if (it != mid.end()) return it->second;
      V3 c = 0.5 * (P[a] + P[b]);
      P.push_back((radius / norm(c)) * c);
      int32_t id = (int32_t)P.size() - 1;
      mid.emplace(key, id);
      return id;
    };
    std::vector<int32_t> T2;
    T2.reserve(4 * T.size());
    for (size_t f = 0; f < T.size(); f += 3) {
      int32_t a = T[f], b = T[f + 1], c = T[f + 2];
      int32_t ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
      const int32_t kids[12] = {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca};
      T2.insert(T2.end(), kids, kids + 12);
    }
    T.swap(T2);
  }
  m.xyz.resize(3 * P.size());
  for (size_t i = 0; i < P.size(); i++) {
    m.xyz[3 * i] = P[i].x;
    m.xyz[3 * i + 1] = P[i].y;
    m.xyz[3 * i + 2] = P[i].z;
  }
  // counter-clockwise seen from outside
  for (size_t f = 0; f < T.size(); f += 3) {
    V3 a = P[T[f]], b = P[T[f + 1]], c = P[T[f + 2]];
    if (dot(cross(b - a, c - a), a + b + c) < 0) std::swap(T[f + 1], T[f + 2]);
  }
  m.tri = T;
  const int nc = (int)T.size() / 3;
  m.cedge.assign(3 * nc, -1);
  m.csgn.assign(3 * nc, 0);
  std::unordered_map<uint64_t, int32_t> eid;
  eid.reserve(2 * T.size());
  for (int c = 0; c < nc; c++)
    for (int i = 0; i < 3; i++) {
      int32_t a = T[3 * c + (i + 1) % 3], b = T[3 * c + (i + 2) % 3];
      uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
      auto it = eid.find(key);
      if (it == eid.end()) {  // first (lower-numbered) cell owns the normal
        int32_t e = (int32_t)m.ecell.size() / 2;
        eid.emplace(key, e);
        m.ecell.push_back(c);
        m.ecell.push_back(-1);
        m.evert.push_back(a);
        m.evert.push_back(b);
        m.cedge[3 * c + i] = e;
        m.csgn[3 * c + i] = 1;
      } else {
        m.ecell[2 * it->second + 1] = c;
        m.cedge[3 * c + i] = it->second;
        m.csgn[3 * c + i] = -1;
      }
    }
  for (int e = 0; e < m.ne(); e++)
    if (m.ecell[2 * e + 1] < 0) throw Error(PA_EINVAL, "mesh is not closed");
  return m;
}

void mass_spectrum(pa_ops *o, int steps, double *lmin, double *lmax);
void build_row_parts(pa_ops *o);

namespace {

double coriolis(double omega, V3 x) { return 2.0 * omega * x.z / norm(x); }

}  // namespace

namespace {
// The nonlinear cell term C_i (Sec. 2.5: volume, kinetic-energy and facet
// integrals of the cell's share of the velocity right-hand side of test
// function i) in terms of the cell's edge fluxes U_0..U_2.  With
// phi_l(x) = s_l/(2A) (x - p_l), u = sum_l U_l phi_l and
// q_i(x) = s_i/(2A) (k x u(x)) . (x - p_i):
//   volume + kinetic energy = U^T S_i U, where
//     S_i = sym(V_i) + (s_i/A) K,
//     K_jl = (A/6) sum over side midpoints m of phi_j(m) . phi_l(m),
//     V_i[m][l] = A sum_{j != i} (phi_m(xbar) . (k x grad lambda_j)) G_ijl,
//     G_ijl = s_i/(2A) (k x phi_l(p_j)) . (p_j - p_i)
//   (grad q_i taken from q_i's vertex values, u(xbar) at the centroid);
//   facet of side a = sum_gp utg_gp sum_l H[a][gp][i][l] U_l, where
//     H = -s_a |side a|/2 s_i/(2A) (k x phi_l(x_gp)) . (x_gp - p_i)
//   at the side's Gauss points in the edge's direction, and utg_gp is the
//   upwind tangential velocity there.
// Layout: per i the six coefficients of (U0^2, U1^2, U2^2, U0 U1, U0 U2,
// U1 U2) (cross terms doubled), then H[a][gp][i][l] from offset 18.  g is the
// cell's geometry row (vertices, normal, area, gradients of the barycentric
// coordinates, side lengths), s the cell's edge signs.
void nl_cell_forms(const double *g, const int s[3], double *out) {
  V3 p[3], gl[3];
  for (int i = 0; i < 3; i++) {
    p[i] = {g[3 * i], g[3 * i + 1], g[3 * i + 2]};
    gl[i] = {g[13 + 3 * i], g[14 + 3 * i], g[15 + 3 * i]};
  }
  const V3 k = {g[9], g[10], g[11]};
  const double A = g[12];
  auto phi = [&](int l, V3 x) { return (s[l] / (2.0 * A)) * (x - p[l]); };
  double K[3][3];
  for (int j = 0; j < 3; j++)
    for (int l = 0; l < 3; l++) {
      double v = 0.0;
      for (int q = 0; q < 3; q++) {
        const V3 mq = 0.5 * (p[(q + 1) % 3] + p[(q + 2) % 3]);
        v += dot(phi(j, mq), phi(l, mq));
      }
      K[j][l] = A / 6.0 * v;
    }
  const V3 xb = (1.0 / 3.0) * (p[0] + p[1] + p[2]);
  for (int i = 0; i < 3; i++) {
    double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < 3; j++) {
      if (j == i) continue;
      const V3 kg = cross(k, gl[j]);
      for (int m = 0; m < 3; m++) {
        const double a = A * dot(phi(m, xb), kg);
        for (int l = 0; l < 3; l++)
          V[m][l] += a * (s[i] / (2.0 * A)) * dot(cross(k, phi(l, p[j])), p[j] - p[i]);
      }
    }
    double S[3][3];
    for (int m = 0; m < 3; m++)
      for (int l = 0; l < 3; l++) S[m][l] = 0.5 * (V[m][l] + V[l][m]) + (s[i] / A) * K[m][l];
    double *o = out + 6 * i;
    o[0] = S[0][0];
    o[1] = S[1][1];
    o[2] = S[2][2];
    o[3] = 2.0 * S[0][1];
    o[4] = 2.0 * S[0][2];
    o[5] = 2.0 * S[1][2];
  }
  const double gq = 0.5 / std::sqrt(3.0);
  for (int a = 0; a < 3; a++) {
    // the side's vertices in the edge's direction (the cell's CCW order when s = +1)
    const int ia = s[a] > 0 ? (a + 1) % 3 : (a + 2) % 3;
    const int ib = s[a] > 0 ? (a + 2) % 3 : (a + 1) % 3;
    for (int gp = 0; gp < 2; gp++) {
      const double xi = gp == 0 ? 0.5 - gq : 0.5 + gq;
      const V3 xg = p[ia] + xi * (p[ib] - p[ia]);
      for (int i = 0; i < 3; i++)
        for (int l = 0; l < 3; l++)
          out[18 + ((2 * a + gp) * 3 + i) * 3 + l] =
              -s[a] * 0.5 * g[22 + a] * (s[i] / (2.0 * A)) * dot(cross(k, phi(l, xg)), xg - p[i]);
    }
  }
}
}  // namespace

// Assemble operators and geometry tables on the host.
void assemble_ops(pa_ops *o, const Mesh &m, const pa_phys &ph) {
  const int ne = m.ne(), nc = m.nc();
  o->ne = ne;
  o->nc = nc;
  o->g = ph.g;
  o->H = ph.H;
  o->omega = ph.omega;
  o->lambda_bar = ph.lambda_bar;
  o->area.resize(nc);
  o->inv_area.resize(nc);
  o->bottom.assign(nc, 0.0);
  if (ph.b_cell) std::memcpy(o->bottom.data(), ph.b_cell, sizeof(double) * nc);
  o->cgeo.assign((size_t)nc * kCellGeo, 0.0);
  o->nlform.assign((size_t)nc * kNlForm, 0.0);
  o->cedge = m.cedge;
  o->csgn = m.csgn;
  o->ecell = m.ecell;
  o->cnbr.resize(3 * nc);
  o->cidx.resize(2 * ne);
  o->cell_edges.resize(12 * nc);
  o->tau.resize((size_t)kEdgeTau * ne);
  o->ell_col.assign(5 * ne, -1);
  o->mass.assign(5 * ne, 0.0);
  o->cor.assign(5 * ne, 0.0);
  o->graddiv.assign(5 * ne, 0.0);

  // ELL pattern: self, then the other two edges of c0, then those of c1
  for (int e = 0; e < ne; e++) {
    o->ell_col[5 * e] = e;
    for (int side = 0; side < 2; side++) {
      int c = m.ecell[2 * e + side], slot = 1 + 2 * side;
      for (int j = 0; j < 3; j++) {
        int ej = m.cedge[3 * c + j];
        if (ej == e) {
          o->cidx[2 * e + side] = 3 * c + j;
        } else {
          o->ell_col[5 * e + slot++] = ej;
        }
      }
    }
  }
  auto ell_slot = [&](int row, int col) {
    for (int j = 0; j < 5; j++)
      if (o->ell_col[5 * row + j] == col) return 5 * row + j;
    throw Error(PA_EINVAL, "ELL pattern mismatch");
  };

  for (int c = 0; c < nc; c++) {
    V3 p[3];
    int s[3], ed[3];
    for (int i = 0; i < 3; i++) {
      p[i] = vert(m, m.tri[3 * c + i]);
      s[i] = m.csgn[3 * c + i];
      ed[i] = m.cedge[3 * c + i];
      int e = ed[i];
      o->cnbr[3 * c + i] = m.ecell[2 * e] == c ? m.ecell[2 * e + 1] : m.ecell[2 * e];
      o->cell_edges[12 * c + i] = e;
      for (int j = 0; j < 3; j++) o->cell_edges[12 * c + 3 + 3 * i + j] = m.cedge[3 * o->cnbr[3 * c + i] + j];
    }
    V3 kk = cross(p[1] - p[0], p[2] - p[0]);
    double A = 0.5 * norm(kk);
    V3 k = (1.0 / (2.0 * A)) * kk;
    o->area[c] = A;
    o->inv_area[c] = 1.0 / A;
    // mass: int (x - p_i).(x - p_j) = A/12 (sum_v f_v.g_v + (sum f).(sum g))
    V3 sumv = p[0] + p[1] + p[2];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double sv = 0;
        for (int v = 0; v < 3; v++) sv += dot(p[v] - p[i], p[v] - p[j]);
        double I = A / 12.0 * (sv + dot(sumv - 3.0 * p[i], sumv - 3.0 * p[j]));
        o->mass[ell_slot(ed[i], ed[j])] += s[i] * s[j] * I / (4.0 * A * A);
      }
    // grad-div D' A^-1 D (the depth elimination of the rational form's
    // shifted systems): s_i s_j / A for every pair of the cell's edges
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) o->graddiv[ell_slot(ed[i], ed[j])] += s[i] * s[j] / A;
    // Coriolis: midpoints of the sides, weight A/3
    for (int q = 0; q < 3; q++) {
      V3 x = 0.5 * (p[(q + 1) % 3] + p[(q + 2) % 3]);
      double fw = coriolis(ph.omega, x) * A / 3.0 / (4.0 * A * A);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          if (i == j) continue;
          double v = dot(k, cross(x - p[j], x - p[i]));  // (x-p_i).(k x (x-p_j))
          o->cor[ell_slot(ed[i], ed[j])] += s[i] * s[j] * fw * v;
        }
    }
    // geometry for the nonlinear kernels
    double *g = &o->cgeo[(size_t)c * kCellGeo];
    for (int i = 0; i < 3; i++) {
      g[3 * i] = p[i].x;
      g[3 * i + 1] = p[i].y;
      g[3 * i + 2] = p[i].z;
    }
    g[9] = k.x;
    g[10] = k.y;
    g[11] = k.z;
    g[12] = A;
    for (int j = 0; j < 3; j++) {  // grad lambda_j = k x (p_{j+2} - p_{j+1}) / 2A
      V3 gl = (1.0 / (2.0 * A)) * cross(k, p[(j + 2) % 3] - p[(j + 1) % 3]);
      g[13 + 3 * j] = gl.x;
      g[14 + 3 * j] = gl.y;
      g[15 + 3 * j] = gl.z;
      g[22 + j] = norm(p[(j + 2) % 3] - p[(j + 1) % 3]);
    }
    nl_cell_forms(g, s, &o->nlform[(size_t)c * kNlForm]);
  }
  // tangential traces t_e . u_c(x_g) = sum_j tau[side][g][j] U_j, at the two
  // Gauss points of the edge taken in the edge's a -> b order
  const double gq = 0.5 / std::sqrt(3.0);
  for (int e = 0; e < ne; e++) {
    V3 a = vert(m, m.evert[2 * e]), b = vert(m, m.evert[2 * e + 1]);
    V3 te = (1.0 / norm(b - a)) * (b - a);
    for (int side = 0; side < 2; side++) {
      int c = m.ecell[2 * e + side];
      const double *g = &o->cgeo[(size_t)c * kCellGeo];
      for (int gp = 0; gp < 2; gp++) {
        V3 x = a + (gp == 0 ? 0.5 - gq : 0.5 + gq) * (b - a);
        for (int j = 0; j < 3; j++) {
          V3 pj = {g[3 * j], g[3 * j + 1], g[3 * j + 2]};
          o->tau[(size_t)kEdgeTau * e + 6 * side + 3 * gp + j] =
              m.csgn[3 * c + j] * dot(te, x - pj) / (2.0 * g[12]);
        }
      }
    }
  }
  o->dinv.resize(ne);
  o->dinv32.resize(ne);
  o->mass32.resize(5 * ne);
  for (int e = 0; e < ne; e++) {
    o->dinv[e] = 1.0 / o->mass[5 * e];
    o->dinv32[e] = (float)o->dinv[e];
  }
  for (int i = 0; i < 5 * ne; i++) o->mass32[i] = (float)o->mass[i];
  build_row_parts(o);
  mass_spectrum(o, 200, &o->mass_eig_min, &o->mass_eig_max);
}

// Row parts of the edge mass matrix for the fused-step solve kernel: rings
// 1..kFusedMax-1 of each part (ELL columns of the previous ring, or of the
// part, outside the part and the earlier rings; ascending within a ring) and
// every ELL column of the part's rows and of its rings 1..kFusedMax-2 as an
// index into the part's local numbering (part rows, then the rings in order).
// A mesh whose rings do not fit kHaloMax rows keeps fewer rings.
void build_row_parts(pa_ops *o) {
  const int ne = o->ne, P = (ne + kPartRows - 1) / kPartRows;
  std::vector<std::vector<int32_t>> rings((size_t)P * (kFusedMax - 1));
  int fmax = kFusedMax;
  std::vector<uint8_t> mark(ne, 0);
  for (int p = 0; p < P; p++) {
    const int e0 = p * kPartRows, e1 = std::min(ne, e0 + kPartRows);
    std::vector<int32_t> front;
    for (int e = e0; e < e1; e++) {
      mark[e] = 1;
      front.push_back(e);
    }
    int total = 0;
    std::vector<int32_t> touched(front);
    for (int r = 0; r < kFusedMax - 1; r++) {
      std::vector<int32_t> &ring = rings[(size_t)p * (kFusedMax - 1) + r];
      for (int e : front)
        for (int j = 0; j < 5; j++) {
          const int c = o->ell_col[5 * e + j];
          if (!mark[c]) {
            mark[c] = 1;
            ring.push_back(c);
          }
        }
      std::sort(ring.begin(), ring.end());
      touched.insert(touched.end(), ring.begin(), ring.end());
      total += (int)ring.size();
      if (total > kHaloMax) fmax = std::min(fmax, r + 1);
      front = ring;
    }
    for (int e : touched) mark[e] = 0;
  }
  // one workgroup per part, and per-workgroup partials for the residual check
  if ((P + 7) / 8 * 8 > launch_max_wg()) fmax = 1;
  o->fused_max = fmax;
  o->hparts = fmax >= 2 ? P : 0;
  // a set-up launch also forms the depth rows: nc / parts per workgroup
  o->fused_cpp = o->hparts ? (o->nc + P - 1) / P : 0;
  if (o->fused_cpp > kPartRows) o->fused_cpp = 0;
  o->ring_cnt.assign((size_t)P * 8, 0);
  o->ring_row.assign((size_t)P * kHaloMax, -1);  // -1: past the part's rings
  o->ring_loc.assign((size_t)P * kHaloMax * 5, 0);
  o->hloc.assign((size_t)5 * ne, 0);
  if (!o->hparts) return;
  std::unordered_map<int32_t, int> loc;
  for (int p = 0; p < P; p++) {
    const int e0 = p * kPartRows, e1 = std::min(ne, e0 + kPartRows);
    loc.clear();
    for (int e = e0; e < e1; e++) loc[e] = e - e0;
    int n = 0;
    for (int r = 0; r < fmax - 1; r++) {
      for (int c : rings[(size_t)p * (kFusedMax - 1) + r]) {
        o->ring_row[(size_t)p * kHaloMax + n] = c;
        loc[c] = kPartRows + n;
        n++;
      }
      o->ring_cnt[(size_t)p * 8 + r] = n;
    }
    for (int r = fmax - 1; r < kFusedMax - 1; r++) o->ring_cnt[(size_t)p * 8 + r] = n;
    for (int S = 2; S <= fmax; S++)
      for (int st = 0; st + 1 < S; st++) {
        const int c = o->ring_cnt[(size_t)p * 8 + S - 2 - st];
        int &sl = o->fused_slots[S][st];
        sl = std::max(sl, (c + kPartRows - 1) / kPartRows);
      }
    for (int e = e0; e < e1; e++)
      for (int j = 0; j < 5; j++) o->hloc[(size_t)j * ne + e] = (uint16_t)loc.at(o->ell_col[5 * e + j]);
    // rings whose rows take later steps: all but the outermost kept ring
    const int inner = fmax >= 3 ? o->ring_cnt[(size_t)p * 8 + fmax - 3] : 0;
    for (int h = 0; h < inner; h++) {
      const int g = o->ring_row[(size_t)p * kHaloMax + h];
      for (int j = 0; j < 5; j++)
        o->ring_loc[((size_t)p * kHaloMax + h) * 5 + j] = (uint16_t)loc.at(o->ell_col[5 * g + j]);
    }
  }
}

namespace {
// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
// (Sturm sequence count).
int sturm_count(const std::vector<double> &al, const std::vector<double> &be, double x) {
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < al.size(); i++) {
    const double b2 = i ? be[i - 1] * be[i - 1] : 0.0;
    d = al[i] - x - (i ? b2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) cnt++;
  }
  return cnt;
}
}  // namespace

// Ritz bounds of a symmetric operator S (y = S x) by Lanczos from a fixed
// start vector, eigenvalues of the tridiagonal matrix by bisection.  The
// Ritz values lie inside the spectrum and approach its ends quickly; callers
// widen them by a margin.
void ritz_bounds(int n, const std::function<void(const std::vector<double> &, std::vector<double> &)> &S,
                 int steps, double *lmin, double *lmax) {
  std::vector<double> v(n), vp(n, 0.0), w(n);
  double nv = 0.0;
  for (int i = 0; i < n; i++) {
    v[i] = 1.0 + 0.5 * std::sin(0.7 * i + 0.3);
    nv += v[i] * v[i];
  }
  nv = std::sqrt(nv);
  for (auto &x : v) x /= nv;
  std::vector<double> al, be;
  double bprev = 0.0;
  for (int k = 0; k < steps; k++) {
    S(v, w);
    double a = 0.0;
    for (int i = 0; i < n; i++) a += w[i] * v[i];
    double b = 0.0;
    for (int i = 0; i < n; i++) {
      w[i] -= a * v[i] + bprev * vp[i];
      b += w[i] * w[i];
    }
    b = std::sqrt(b);
    al.push_back(a);
    if (b < 1e-14 || k + 1 == steps) break;
    be.push_back(b);
    for (int i = 0; i < n; i++) {
      vp[i] = v[i];
      v[i] = w[i] / b;
    }
    bprev = b;
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  double lo = 1e300, hi = -1e300;  // Gershgorin interval of T
  for (size_t i = 0; i < al.size(); i++) {
    const double r = (i ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < al.size() ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto kth = [&](int k) {  // k-th smallest eigenvalue of T (0-based)
    double a = lo, b = hi;
    for (int it = 0; it < 200; it++) {
      const double m = 0.5 * (a + b);
      if (sturm_count(al, be, m) > k) b = m; else a = m;
    }
    return 0.5 * (a + b);
  };
  *lmin = kth(0);
  *lmax = kth((int)al.size() - 1);
}

// Extreme eigenvalues of D^-1 M, through its symmetric form D^-1/2 M D^-1/2.
void mass_spectrum(pa_ops *o, int steps, double *lmin, double *lmax) {
  const int n = o->ne;
  std::vector<double> sq(n);
  for (int i = 0; i < n; i++) sq[i] = std::sqrt(o->dinv[i]);
  ritz_bounds(
      n,
      [&](const std::vector<double> &v, std::vector<double> &w) {
        for (int i = 0; i < n; i++) {
          double s = 0.0;
          for (int j = 0; j < 5; j++) {
            const int c = o->ell_col[5 * i + j];
            s += o->mass[5 * i + j] * sq[c] * v[c];
          }
          w[i] = sq[i] * s;
        }
      },
      steps, lmin, lmax);
}

// Chebyshev weights of exp(i theta x): (2 - delta_k0) J_k(theta), k = 0..kcap,
// J_k by Miller's downward recurrence J_{k-1} = (2k/theta) J_k - J_{k+1},
// normalised with J_0 + 2 sum_m J_2m = 1.
std::vector<double> bessel_weights(double theta, int kcap) {
  std::vector<double> c(kcap + 1, 0.0);
  if (theta == 0.0) {
    c[0] = 1.0;
    return c;
  }
  int start = kcap + 20 + (int)(2.0 * theta) + 2 * (int)std::sqrt(40.0 * (kcap + theta));
  start += start & 1;
  std::vector<double> J(start + 2, 0.0);
  J[start + 1] = 0.0;
  J[start] = 1e-300;
  double norm = 0.0;
  for (int k = start; k >= 1; k--) {
    J[k - 1] = (2.0 * k / theta) * J[k] - J[k + 1];
    if (std::fabs(J[k - 1]) > 1e250) {  // rescale to avoid overflow
      for (int j = k - 1; j <= start + 1; j++) J[j] *= 1e-250;
      norm *= 1e-250;
    }
    if ((k - 1) % 2 == 0 && k - 1 > 0) norm += 2.0 * J[k - 1];
  }
  norm += J[0];
  for (int k = 0; k <= kcap; k++) c[k] = (k == 0 ? 1.0 : 2.0) * J[k] / norm;
  return c;
}

// Smallest K with sum_{k>K} |c_k| <= tol (drop from the top while the
// dropped magnitude stays within tol).
int truncate_degree(const std::vector<double> &c, double tol) {
  double tail = 0.0;
  int K = (int)c.size() - 1;
  while (K > 0 && tail + std::fabs(c[K]) <= tol) {
    tail += std::fabs(c[K]);
    K--;
  }
  return K;
}

}  // namespace pa
