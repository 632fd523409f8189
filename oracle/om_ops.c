/*
 * Oracle: the discrete linear operator L of the paper's Sec. 2.5, written for
 * the RT0/P0 pair, its velocity mass solve, and a power-iteration estimate of
 * its spectral radius.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Weak form (Sec. 2.5, the discrete linear operator):
 *   int w . u1 = - int w . (f u^perp) + int (div w) g eta      for all w in V1
 *   int phi eta1 = - H int phi div u                           for all phi in V2
 * with u^perp = k x u (Sec. 2.1).  For RT0 on a flat triangle T the basis
 * function of local edge i is s_i (x - p_i) / (2|T|), where p_i is the vertex
 * opposite edge i and s_i = +1 when the global edge normal points out of T;
 * its flux through edge i is s_i and its divergence is s_i / |T|.
 * Integrals over T use the edge-midpoint rule, exact for quadratics.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

void om_cell_geom(const struct om_mesh *m, int c, om_cell *T) {
  for (int i = 0; i < 3; i++) {
    memcpy(T->p[i], m->x + 3 * m->cv[3 * c + i], 3 * sizeof(double));
    T->s[i] = m->csign[3 * c + i];
    T->e[i] = m->ce[3 * c + i];
  }
  double e1[3], e2[3], k[3];
  om_sub(T->p[1], T->p[0], e1);
  om_sub(T->p[2], T->p[0], e2);
  om_cross(e1, e2, k);
  double nk = sqrt(om_dot(k, k));
  T->area = 0.5 * nk;
  for (int d = 0; d < 3; d++) T->k[d] = k[d] / nk;
}

void om_rt0_basis(const om_cell *T, int i, const double *x, double *phi) {
  double f = T->s[i] / (2.0 * T->area);
  for (int d = 0; d < 3; d++) phi[d] = f * (x[d] - T->p[i][d]);
}

void om_rt0_velocity(const om_cell *T, const double *U, const double *x, double *u) {
  u[0] = u[1] = u[2] = 0;
  for (int j = 0; j < 3; j++) {
    double phi[3];
    om_rt0_basis(T, j, x, phi);
    for (int d = 0; d < 3; d++) u[d] += U[T->e[j]] * phi[d];
  }
}

/* Coriolis parameter f = 2 Omega sin(latitude) at a point. */
static double coriolis(double Omega, const double *x) {
  return 2.0 * Omega * x[2] / sqrt(om_dot(x, x));
}

/* Add value v at (r, c) of a CSR matrix whose rows have room for 'cap'
 * entries; rows are filled in insertion order. */
static void csr_add(int *cnt, int *col, double *v1, double *v2, int cap, int r,
                    int c, double a1, double a2) {
  for (int j = 0; j < cnt[r]; j++)
    if (col[cap * r + j] == c) {
      v1[cap * r + j] += a1;
      v2[cap * r + j] += a2;
      return;
    }
  int j = cnt[r]++;
  if (j >= cap) abort();
  col[cap * r + j] = c;
  v1[cap * r + j] = a1;
  v2[cap * r + j] = a2;
}

om_ops *om_ops_create(const om_mesh *m, double g, double H, double Omega,
                      const double *b_cell) {
  om_ops *o = calloc(1, sizeof(om_ops));
  o->m = m;
  o->g = g;
  o->H = H;
  o->Omega = Omega;
  int ne = m->ne, nc = m->nc;
  o->b = calloc(nc, sizeof(double));
  if (b_cell) memcpy(o->b, b_cell, sizeof(double) * nc);
  o->area = malloc(sizeof(double) * nc);
  const int cap = 8;
  int *cnt = calloc(ne, sizeof(int));
  int *col = malloc(sizeof(int) * cap * ne);
  double *vm = calloc((size_t)cap * ne, sizeof(double));
  double *vf = calloc((size_t)cap * ne, sizeof(double));
  for (int c = 0; c < nc; c++) {
    om_cell T;
    om_cell_geom(m, c, &T);
    o->area[c] = T.area;
    double mloc[3][3] = {{0}}, floc[3][3] = {{0}};
    for (int q = 0; q < 3; q++) {
      /* midpoint of the edge opposite vertex q, weight |T|/3 */
      double x[3];
      for (int d = 0; d < 3; d++)
        x[d] = 0.5 * (T.p[(q + 1) % 3][d] + T.p[(q + 2) % 3][d]);
      double wq = T.area / 3.0, f = coriolis(Omega, x);
      double phi[3][3], kphi[3][3];
      for (int i = 0; i < 3; i++) {
        om_rt0_basis(&T, i, x, phi[i]);
        om_cross(T.k, phi[i], kphi[i]);
      }
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
          mloc[i][j] += wq * om_dot(phi[i], phi[j]);
          floc[i][j] += wq * f * om_dot(phi[i], kphi[j]);
        }
    }
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        csr_add(cnt, col, vm, vf, cap, T.e[i], T.e[j], mloc[i][j], floc[i][j]);
  }
  o->rowptr = malloc(sizeof(int) * (ne + 1));
  o->rowptr[0] = 0;
  for (int r = 0; r < ne; r++) o->rowptr[r + 1] = o->rowptr[r] + cnt[r];
  o->nnz = o->rowptr[ne];
  o->col = malloc(sizeof(int) * o->nnz);
  o->mass = malloc(sizeof(double) * o->nnz);
  o->cor = malloc(sizeof(double) * o->nnz);
  o->diag = malloc(sizeof(double) * ne);
  for (int r = 0; r < ne; r++)
    for (int j = 0; j < cnt[r]; j++) {
      int k = o->rowptr[r] + j;
      o->col[k] = col[cap * r + j];
      o->mass[k] = vm[cap * r + j];
      o->cor[k] = vf[cap * r + j];
      if (o->col[k] == r) o->diag[r] = o->mass[k];
    }
  free(cnt); free(col); free(vm); free(vf);
  return o;
}

void om_ops_destroy(om_ops *o) {
  if (!o) return;
  free(o->b); free(o->area); free(o->rowptr); free(o->col);
  free(o->mass); free(o->cor); free(o->diag);
  free(o);
}

int om_ops_export(const om_ops *o, int32_t *rowptr, int32_t *cols, double *mass,
                  double *cor, double *area) {
  int ne = o->m->ne;
  if (rowptr) for (int i = 0; i <= ne; i++) rowptr[i] = o->rowptr[i];
  for (int k = 0; k < o->nnz; k++) {
    if (cols) cols[k] = o->col[k];
    if (mass) mass[k] = o->mass[k];
    if (cor) cor[k] = o->cor[k];
  }
  if (area) memcpy(area, o->area, sizeof(double) * o->m->nc);
  return o->nnz;
}

static void spmv(const om_ops *o, const double *val, const double *x, double *y) {
  for (int r = 0; r < o->m->ne; r++) {
    double s = 0;
    for (int k = o->rowptr[r]; k < o->rowptr[r + 1]; k++) s += val[k] * x[o->col[k]];
    y[r] = s;
  }
}

static double dot(const double *a, const double *b, int n) {
  double s = 0;
  for (int i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

int om_mass_solve(const om_ops *o, const double *b, double *x, double rtol, int maxit) {
  int n = o->m->ne;
  double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
  double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
  for (int i = 0; i < n; i++) {
    x[i] = 0;
    r[i] = b[i];
    z[i] = r[i] / o->diag[i];
    p[i] = z[i];
  }
  double bnorm = sqrt(dot(b, b, n)), rz = dot(r, z, n);
  int it = 0, status = -1;
  if (bnorm == 0.0) status = 0;
  while (status < 0 && it < maxit) {
    spmv(o, o->mass, p, q);
    double alpha = rz / dot(p, q, n);
    for (int i = 0; i < n; i++) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    it++;
    if (sqrt(dot(r, r, n)) <= rtol * bnorm) {
      status = it;
      break;
    }
    for (int i = 0; i < n; i++) z[i] = r[i] / o->diag[i];
    double rz_new = dot(r, z, n);
    double beta = rz_new / rz;
    rz = rz_new;
    for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
  }
  free(r); free(z); free(p); free(q);
  return status;
}

int om_apply_L(const om_ops *o, const double *U, double *out, double rtol) {
  const om_mesh *m = o->m;
  int ne = m->ne, nc = m->nc;
  const double *u = U, *eta = U + ne;
  double *rhs = malloc(sizeof(double) * ne);
  /* velocity: int w . u1 = -int w.(f u^perp) + g int (div w) eta.  The last
   * term is g * s_{T,i} * eta_T summed over the two cells of edge i. */
  spmv(o, o->cor, u, rhs);
  for (int i = 0; i < ne; i++) rhs[i] = -rhs[i];
  for (int c = 0; c < nc; c++)
    for (int i = 0; i < 3; i++)
      rhs[m->ce[3 * c + i]] += o->g * m->csign[3 * c + i] * eta[c];
  int it = om_mass_solve(o, rhs, out, rtol, 1000);
  /* depth: |T| eta1 = -H * (outward flux of u through the sides of T) */
  for (int c = 0; c < nc; c++) {
    double div = 0;
    for (int i = 0; i < 3; i++) div += m->csign[3 * c + i] * u[m->ce[3 * c + i]];
    out[ne + c] = -o->H * div / o->area[c];
  }
  free(rhs);
  return it < 0 ? -1 : 0;
}

/* W inner product <X, Y>_W = H u_X' M u_Y + g sum_c |c| eta_X eta_Y, in
 * which L is skew-adjoint. */
static double wdot(const om_ops *o, const double *X, const double *Y) {
  int ne = o->m->ne, nc = o->m->nc;
  double *q = malloc(sizeof(double) * ne);
  spmv(o, o->mass, Y, q);
  double s = o->H * dot(X, q, ne);
  for (int c = 0; c < nc; c++) s += o->g * o->area[c] * X[ne + c] * Y[ne + c];
  free(q);
  return s;
}

double om_power_rho(const om_ops *o, const double *v0, int iters, double rtol) {
  int n = o->m->ne + o->m->nc;
  double *v = malloc(sizeof(double) * n), *a = malloc(sizeof(double) * n);
  double *b = malloc(sizeof(double) * n);
  memcpy(v, v0, sizeof(double) * n);
  double rho2 = 0;
  for (int it = 0; it < iters; it++) {
    double nv = sqrt(wdot(o, v, v));
    for (int i = 0; i < n; i++) v[i] /= nv;
    om_apply_L(o, v, a, rtol);
    /* <v, -L^2 v>_W = <L v, L v>_W since L is W-skew */
    rho2 = wdot(o, a, a);
    om_apply_L(o, a, b, rtol);
    for (int i = 0; i < n; i++) v[i] = -b[i];
  }
  free(v); free(a); free(b);
  return sqrt(rho2);
}

void om_diagnostics(const om_ops *o, const double *U, double *out) {
  const om_mesh *m = o->m;
  int ne = m->ne, nc = m->nc;
  const double *u = U, *eta = U + ne;
  double *q = malloc(sizeof(double) * ne);
  spmv(o, o->mass, u, q);
  double uMu = dot(u, q, ne);
  double mass = 0, e2 = 0, div2 = 0, ke = 0;
  for (int c = 0; c < nc; c++) {
    mass += o->area[c] * eta[c];
    e2 += o->area[c] * eta[c] * eta[c];
    double div = 0;
    for (int i = 0; i < 3; i++) div += m->csign[3 * c + i] * u[m->ce[3 * c + i]];
    div2 += div * div / o->area[c];
    /* int_T 1/2 h |u|^2 with h = H + eta - b constant on the cell */
    om_cell T;
    om_cell_geom(m, c, &T);
    double s = 0;
    for (int qd = 0; qd < 3; qd++) {
      double x[3], uu[3];
      for (int d = 0; d < 3; d++)
        x[d] = 0.5 * (T.p[(qd + 1) % 3][d] + T.p[(qd + 2) % 3][d]);
      om_rt0_velocity(&T, u, x, uu);
      s += T.area / 3.0 * 0.5 * om_dot(uu, uu);
    }
    ke += (o->H + eta[c] - o->b[c]) * s;
  }
  out[0] = mass;
  out[1] = 0.5 * (o->H * uMu + o->g * e2);
  out[2] = ke + 0.5 * o->g * e2;
  out[3] = sqrt(uMu + div2);
  out[4] = sqrt(e2);
  free(q);
}
