/*
 * Oracle: phase averaging (Sec. 2.2) and the averaged Lawson RK4 step
 * (Sec. 2.3).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Averaged nonlinearity (eq. vt_discretised):
 *   Nbar(U) = sum_m w_m exp(-s_m L) N(exp(s_m L) U),
 * every term evaluated on its own, accumulated in node order in FP64, with
 * the exponential either the Chebyshev polynomial of Sec. 2.4 or the
 * rational (REXI) sum of om_rexi.c.
 *
 * Readings of the averaging formula (eq. vt_averaged and the weight rho):
 *  - rho is the standard smooth bump exp(-1/(1/4 - sigma^2)) on |sigma| < 1/2
 *    (the printed exponent has the opposite sign, which grows towards the
 *    ends of the interval instead of vanishing);
 *  - the weights are normalised discretely to sum to one, which is what the
 *    T -> 0 limit (the unaveraged equation) requires;
 *  - the nodes are the M midpoints of the support of rho(s/T), s in
 *    (-T/2, T/2), spacing T/M; the printed nodes kT/N over [-T, T] would put
 *    half of them where the weight vanishes.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

void om_avg_nodes(int M, double T, double *s, double *w) {
  double sum = 0;
  for (int m = 0; m < M; m++) {
    double sigma = -0.5 + (m + 0.5) / M;
    s[m] = T * sigma;
    w[m] = exp(-1.0 / (0.25 - sigma * sigma));
    sum += w[m];
  }
  for (int m = 0; m < M; m++) w[m] /= sum;
}

/* Which construction of exp(t L) the averaging and the step use: the
 * Chebyshev polynomial (Sec. 2.4, truncation threshold tol) or the rational
 * (REXI) sum with N nodes on the ellipse of parameter eta0, each shifted
 * system solved by GMRES to gm_rtol (om_rexi.c). */
typedef struct {
  int rexi, N;
  double tol, eta0, gm_rtol;
} expo_cfg;

static int expo(const om_ops *o, const expo_cfg *ec, double lb, double t, double rtol,
                const double *U, double *out) {
  if (ec->rexi) return om_rexi_expL(o, lb, t, ec->N, ec->eta0, ec->gm_rtol, rtol, U, out);
  return om_expL(o, lb, t, ec->tol, rtol, U, out);
}

static int inner_op(const om_ops *o, int which_n, const double *X, double *Y,
                    double rtol) {
  int n = o->m->ne + o->m->nc;
  if (which_n == 1) {
    memcpy(Y, X, sizeof(double) * n);
    return 0;
  }
  if (which_n == 2) return om_apply_L(o, X, Y, rtol);
  return om_nonlinear(o, X, Y, rtol);
}

static int avg_rhs(const om_ops *o, const expo_cfg *ec, double lambda_bar, int nnodes,
                   const double *s, const double *w, double rtol, int which_n,
                   const double *U, double *out) {
  int n = o->m->ne + o->m->nc;
  double *E = malloc(sizeof(double) * n), *Y = malloc(sizeof(double) * n);
  double *Z = malloc(sizeof(double) * n);
  memset(out, 0, sizeof(double) * n);
  int status = 0;
  for (int m = 0; m < nnodes && status == 0; m++) {
    if (expo(o, ec, lambda_bar, s[m], rtol, U, E) < 0) status = -1;
    if (status == 0 && inner_op(o, which_n, E, Y, rtol) < 0) status = -1;
    if (status == 0 && expo(o, ec, lambda_bar, -s[m], rtol, Y, Z) < 0) status = -1;
    for (int i = 0; i < n; i++) out[i] += w[m] * Z[i];
  }
  free(E); free(Y); free(Z);
  return status;
}

int om_phase_avg_rhs(const om_ops *o, double lambda_bar, int nnodes,
                     const double *s, const double *w, double tol, double rtol,
                     int which_n, const double *U, double *out) {
  expo_cfg ec = {0, 0, tol, 0.0, 0.0};
  return avg_rhs(o, &ec, lambda_bar, nnodes, s, w, rtol, which_n, U, out);
}

int om_rexi_phase_avg_rhs(const om_ops *o, double lambda_bar, int nnodes, const double *s,
                          const double *w, int N, double eta0, double gm_rtol, double rtol,
                          int which_n, const double *U, double *out) {
  expo_cfg ec = {1, N, 0.0, eta0, gm_rtol};
  return avg_rhs(o, &ec, lambda_bar, nnodes, s, w, rtol, which_n, U, out);
}

/* < exp(-L s) N(exp(L dt/2) exp(L s) X) >_s : the bracket with the extra
 * half-step exponential inside N, as written in stages 2 and 4. */
static int bracket_shifted(const om_ops *o, const expo_cfg *ec, double lb, int nn, const double *s,
                           const double *w, double half, double rtol,
                           int which_n, const double *X, double *out) {
  int n = o->m->ne + o->m->nc;
  double *E = malloc(sizeof(double) * n), *E2 = malloc(sizeof(double) * n);
  double *Y = malloc(sizeof(double) * n), *Z = malloc(sizeof(double) * n);
  memset(out, 0, sizeof(double) * n);
  int st = 0;
  for (int m = 0; m < nn && st == 0; m++) {
    if (expo(o, ec, lb, s[m], rtol, X, E) < 0) st = -1;
    if (st == 0 && expo(o, ec, lb, half, rtol, E, E2) < 0) st = -1;
    if (st == 0 && inner_op(o, which_n, E2, Y, rtol) < 0) st = -1;
    if (st == 0 && expo(o, ec, lb, -s[m], rtol, Y, Z) < 0) st = -1;
    for (int i = 0; i < n; i++) out[i] += w[m] * Z[i];
  }
  free(E); free(E2); free(Y); free(Z);
  return st;
}

static int lawson_step(const om_ops *o, const expo_cfg *ec, double lb, int nn,
                       const double *s, const double *w, double dt, double rtol, int which_n,
                       double *U) {
  int n = o->m->ne + o->m->nc;
  size_t sz = sizeof(double) * n;
  double *k1 = malloc(sz), *k2 = malloc(sz), *k3 = malloc(sz), *k4 = malloc(sz);
  double *U1 = malloc(sz), *U2 = malloc(sz), *U3 = malloc(sz), *Eh = malloc(sz);
  double *t1 = malloc(sz), *t2 = malloc(sz);
  int st = 0;
  /* stage 1: U1 = U^n + dt/2 <..(U^n)> */
  st |= avg_rhs(o, ec, lb, nn, s, w, rtol, which_n, U, k1);
  for (int i = 0; i < n; i++) U1[i] = U[i] + 0.5 * dt * k1[i];
  /* stage 2: U2 = exp(L dt/2) U^n + dt/2 <exp(-Ls) N(exp(L dt/2) exp(Ls) U1)> */
  st |= expo(o, ec, lb, 0.5 * dt, rtol, U, Eh) < 0;
  st |= bracket_shifted(o, ec, lb, nn, s, w, 0.5 * dt, rtol, which_n, U1, k2);
  for (int i = 0; i < n; i++) U2[i] = Eh[i] + 0.5 * dt * k2[i];
  /* stage 3: U3 = exp(L dt/2) U^n + dt <..(U2)> */
  st |= avg_rhs(o, ec, lb, nn, s, w, rtol, which_n, U2, k3);
  for (int i = 0; i < n; i++) U3[i] = Eh[i] + dt * k3[i];
  /* stage 4 */
  st |= bracket_shifted(o, ec, lb, nn, s, w, 0.5 * dt, rtol, which_n, U3, k4);
  double *acc = U1; /* reuse */
  st |= expo(o, ec, lb, dt, rtol, U, acc) < 0;        /* exp(L dt) U^n */
  st |= expo(o, ec, lb, dt, rtol, k1, t1) < 0;        /* exp(L dt) k1 */
  for (int i = 0; i < n; i++) acc[i] += dt / 6.0 * t1[i];
  st |= expo(o, ec, lb, 0.5 * dt, rtol, k2, t1) < 0;  /* 2 exp(L dt/2) k2 */
  st |= expo(o, ec, lb, 0.5 * dt, rtol, k3, t2) < 0;  /* 2 exp(L dt/2) k3 */
  for (int i = 0; i < n; i++)
    U[i] = acc[i] + dt / 6.0 * (2.0 * t1[i] + 2.0 * t2[i] + k4[i]);
  free(k1); free(k2); free(k3); free(k4); free(U1); free(U2); free(U3); free(Eh);
  free(t1); free(t2);
  return st ? -1 : 0;
}

int om_step(const om_ops *o, double lb, int nn, const double *s, const double *w,
            double dt, double tol, double rtol, int which_n, double *U) {
  expo_cfg ec = {0, 0, tol, 0.0, 0.0};
  return lawson_step(o, &ec, lb, nn, s, w, dt, rtol, which_n, U);
}

int om_rexi_step(const om_ops *o, double lb, int nn, const double *s, const double *w,
                 double dt, int N, double eta0, double gm_rtol, double rtol, int which_n,
                 double *U) {
  expo_cfg ec = {1, N, 0.0, eta0, gm_rtol};
  return lawson_step(o, &ec, lb, nn, s, w, dt, rtol, which_n, U);
}
