/*
 * Oracle: the discrete nonlinearity N of the paper's Sec. 2.5, for RT0/P0.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * N(u, eta) = (u2, eta2) with, for every test function w in V1, phi in V2,
 *   int w.u2   = int u . grad^perp(u^perp . w) - int_Gamma [[n^perp (u^perp . w)]] . u~
 *                + int (div w) |u|^2 / 2
 *   int phi eta2 = int grad phi . u (eta - b) - int_Gamma [[phi u]] (eta - b)~
 * where u^perp = k x u, grad^perp = k x grad, [[q]] = q+ n+ + q- n- and
 * [[v]] = v+.n+ + v-.n-, and ~ marks the value taken from the upwind side.
 *
 * Readings of the printed formulas (each stated where it is used):
 *  (a) upwind side: the printed inequality picks the side the flow enters
 *      when n+ is the outward normal of the + side; the side the flow leaves
 *      is used (edge flux > 0, i.e. flow out of c0, takes c0; otherwise c1);
 *  (b) the facet term of the depth equation carries a minus sign, which is
 *      what integrating -div(u (eta - b)) by parts cell by cell gives;
 *  (c) the facet value of (eta - b) is the upwind cell value.
 *
 * Evaluation follows the weak form literally: for each velocity test function
 * (edge i) loop over the two cells in its support, integrate the cell terms
 * with the edge-midpoint rule (exact for quadratics) and the facet terms of
 * every side of those cells with two-point Gauss (integrands are quadratic
 * along a side), then solve with the velocity mass matrix.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

/* q(x) = (k x u(x)) . phi_i(x) on cell T */
static double q_test(const om_cell *T, const double *U, int i, const double *x) {
  double u[3], ku[3], phi[3];
  om_rt0_velocity(T, U, x, u);
  om_cross(T->k, u, ku);
  om_rt0_basis(T, i, x, phi);
  return om_dot(ku, phi);
}

/* index of the cell the flow leaves through edge e (reading (a)) */
static int upwind_cell(const om_mesh *m, const double *U, int e) {
  return U[e] > 0 ? m->ec[2 * e] : m->ec[2 * e + 1];
}

/* Velocity right-hand side for test function w = phi of edge ei. */
static double velocity_rhs(const om_ops *o, const double *U, int ei) {
  const om_mesh *m = o->m;
  double r = 0;
  for (int side = 0; side < 2; side++) {
    int c = m->ec[2 * ei + side];
    om_cell T;
    om_cell_geom(m, c, &T);
    int li = -1;
    for (int i = 0; i < 3; i++)
      if (T.e[i] == ei) li = i;
    /* gradient of the affine function q on T from its vertex values:
       grad lambda_j = k x (p_{j+2} - p_{j+1}) / (2|T|) */
    double gq[3] = {0, 0, 0};
    for (int j = 0; j < 3; j++) {
      double qj = q_test(&T, U, li, T.p[j]);
      double side_vec[3], gl[3];
      om_sub(T.p[(j + 2) % 3], T.p[(j + 1) % 3], side_vec);
      om_cross(T.k, side_vec, gl);
      for (int d = 0; d < 3; d++) gq[d] += qj * gl[d] / (2.0 * T.area);
    }
    double gperp[3];
    om_cross(T.k, gq, gperp);
    double divw = T.s[li] / T.area;
    for (int q = 0; q < 3; q++) {
      double x[3], u[3];
      for (int d = 0; d < 3; d++) x[d] = 0.5 * (T.p[(q + 1) % 3][d] + T.p[(q + 2) % 3][d]);
      om_rt0_velocity(&T, U, x, u);
      double wq = T.area / 3.0;
      r += wq * om_dot(u, gperp);             /* int u . grad^perp(u^perp . w) */
      r += wq * divw * 0.5 * om_dot(u, u);    /* int (div w) |u|^2 / 2 */
    }
    /* facet terms: this cell's share of - int [[n^perp (u^perp . w)]] . u~ */
    for (int a = 0; a < 3; a++) {
      const double *A = T.p[(a + 1) % 3], *B = T.p[(a + 2) % 3];
      double t[3], len, nout[3], nperp[3];
      om_sub(B, A, t);
      len = sqrt(om_dot(t, t));
      for (int d = 0; d < 3; d++) t[d] /= len;
      om_cross(t, T.k, nout);    /* outward normal of T on this side */
      om_cross(T.k, nout, nperp);
      int e = T.e[a];
      int cu = upwind_cell(m, U, e);
      om_cell Tu;
      om_cell_geom(m, cu, &Tu);
      const double g = 0.5 / sqrt(3.0);
      for (int gp = 0; gp < 2; gp++) {
        double x[3], uu[3];
        double xi = gp == 0 ? 0.5 - g : 0.5 + g;
        for (int d = 0; d < 3; d++) x[d] = A[d] + xi * (B[d] - A[d]);
        om_rt0_velocity(&Tu, U, x, uu);
        r -= 0.5 * len * om_dot(nperp, uu) * q_test(&T, U, li, x);
      }
    }
  }
  return r;
}

int om_nonlinear(const om_ops *o, const double *U, double *out, double rtol) {
  const om_mesh *m = o->m;
  int ne = m->ne, nc = m->nc;
  const double *eta = U + ne;
  double *rhs = malloc(sizeof(double) * ne);
  for (int i = 0; i < ne; i++) rhs[i] = velocity_rhs(o, U, i);
  int it = om_mass_solve(o, rhs, out, rtol, 1000);
  /* depth: |T| eta2 = - sum over sides of (outward flux) * (eta - b)_upwind */
  for (int c = 0; c < nc; c++) {
    double s = 0;
    for (int a = 0; a < 3; a++) {
      int e = m->ce[3 * c + a];
      int cu = upwind_cell(m, U, e);
      s -= m->csign[3 * c + a] * U[e] * (eta[cu] - o->b[cu]);
    }
    out[ne + c] = s / o->area[c];
  }
  free(rhs);
  return it < 0 ? -1 : 0;
}
