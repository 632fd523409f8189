/*
 * Oracle: the rational (REXI) form of the exponential named in the paper's
 * Sec. 2.4 and Sec. 4 -- a sum of rational functions of L, each term of which
 * needs one complex shifted solve, all terms independent of each other.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper does not fix a construction of the rational function.  The one
 * taken here is the Cauchy integral of exp(i theta X) along a Bernstein
 * ellipse around [-1, 1],
 *     exp(i theta x) = (1 / 2 pi i) oint exp(i theta X) / (X - x) dX,
 *     X(phi) = cosh(eta0 + i phi), 0 <= phi < 2 pi,
 * discretised by the N-point trapezoidal rule at phi_j = 2 pi (j + 1/2) / N
 * (the exponentially convergent trapezoidal rule for periodic analytic
 * integrands; Trefethen & Weideman, SIAM Review 56, 2014):
 *     r(x) = sum_j c_j / (X_j - x),  c_j = exp(i theta X_j) sinh(eta0 + i phi_j) / N.
 * With the operator X = -i L / lambda_bar (spectrum in [-1, 1] when
 * lambda_bar >= rho(L)) and theta = lambda_bar t, exp(t L) = exp(i theta X),
 * so
 *     exp(t L) U ~ sum_j c_j y_j,   (X_j I + (i / lambda_bar) L) y_j = U.
 * N and eta0 are parameters handed in by the caller (as lambda_bar is).
 * Every one of the N shifted systems is solved on its own by GMRES on the
 * operator exactly as written (each application of L one velocity mass
 * solve), and the real part of the sum is returned (the exact sum is real:
 * the nodes come in pairs X, -conj(X) whose terms are complex conjugates).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

void om_rexi_coeffs(double theta, int N, double eta0, double *X, double *c) {
  const double pi = acos(-1.0);
  for (int j = 0; j < N; j++) {
    double phi = 2.0 * pi * (j + 0.5) / N;
    double complex w = eta0 + I * phi;
    double complex Xj = ccosh(w);
    double complex cj = cexp(I * theta * Xj) * csinh(w) / N;
    X[2 * j] = creal(Xj);
    X[2 * j + 1] = cimag(Xj);
    c[2 * j] = creal(cj);
    c[2 * j + 1] = cimag(cj);
  }
}

/* y = (Xs I + (i / lb) L) v for complex v (L is real: applied to the real and
 * imaginary parts separately). */
static int shifted_apply(const om_ops *o, double complex Xs, double lb, const double complex *v,
                         double complex *y, double *re, double *im, double *Lre, double *Lim,
                         double rtol) {
  int n = o->m->ne + o->m->nc;
  for (int i = 0; i < n; i++) {
    re[i] = creal(v[i]);
    im[i] = cimag(v[i]);
  }
  if (om_apply_L(o, re, Lre, rtol) < 0 || om_apply_L(o, im, Lim, rtol) < 0) return -1;
  for (int i = 0; i < n; i++) y[i] = Xs * v[i] + (I / lb) * (Lre[i] + I * Lim[i]);
  return 0;
}

static double cnorm(const double complex *v, int n) {
  double s = 0;
  for (int i = 0; i < n; i++) s += creal(v[i] * conj(v[i]));
  return sqrt(s);
}

/* GMRES (no restart, modified Gram-Schmidt, Givens rotations) for
 * (Xs I + (i / lb) L) y = b from y = 0, stopping when the residual norm is at
 * most gm_rtol ||b||.  Returns the iteration count, -1 on failure. */
static int gmres_shifted(const om_ops *o, double complex Xs, double lb, const double *b,
                         double complex *y, double gm_rtol, double rtol, int maxit) {
  int n = o->m->ne + o->m->nc;
  double complex *V = malloc(sizeof(double complex) * (size_t)n * (maxit + 1));
  double complex *Hm = calloc((size_t)(maxit + 1) * maxit, sizeof(double complex));
  double complex *cs = malloc(sizeof(double complex) * maxit);
  double complex *sn = malloc(sizeof(double complex) * maxit);
  double complex *g = calloc(maxit + 1, sizeof(double complex));
  double *re = malloc(sizeof(double) * n), *im = malloc(sizeof(double) * n);
  double *Lre = malloc(sizeof(double) * n), *Lim = malloc(sizeof(double) * n);
  int status = -1, k = 0;
  double bn = 0;
  for (int i = 0; i < n; i++) bn += b[i] * b[i];
  bn = sqrt(bn);
  for (int i = 0; i < n; i++) y[i] = 0;
  if (bn == 0) {
    status = 0;
    goto done;
  }
  for (int i = 0; i < n; i++) V[i] = b[i] / bn;
  g[0] = bn;
  for (k = 0; k < maxit; k++) {
    double complex *w = V + (size_t)n * (k + 1);
    if (shifted_apply(o, Xs, lb, V + (size_t)n * k, w, re, im, Lre, Lim, rtol) < 0) goto done;
    for (int j = 0; j <= k; j++) {
      const double complex *vj = V + (size_t)n * j;
      double complex h = 0;
      for (int i = 0; i < n; i++) h += conj(vj[i]) * w[i];
      for (int i = 0; i < n; i++) w[i] -= h * vj[i];
      Hm[(size_t)j * maxit + k] = h;
    }
    double hn = cnorm(w, n);
    Hm[(size_t)(k + 1) * maxit + k] = hn;
    if (hn > 0)
      for (int i = 0; i < n; i++) w[i] /= hn;
    /* earlier rotations on the new column, then a rotation zeroing h_{k+1,k} */
    for (int j = 0; j < k; j++) {
      double complex a = Hm[(size_t)j * maxit + k], bb = Hm[(size_t)(j + 1) * maxit + k];
      Hm[(size_t)j * maxit + k] = conj(cs[j]) * a + conj(sn[j]) * bb;
      Hm[(size_t)(j + 1) * maxit + k] = -sn[j] * a + cs[j] * bb;
    }
    double complex a = Hm[(size_t)k * maxit + k];
    double r = sqrt(creal(a * conj(a)) + hn * hn);
    cs[k] = a / r;
    sn[k] = hn / r;
    Hm[(size_t)k * maxit + k] = r;
    Hm[(size_t)(k + 1) * maxit + k] = 0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = conj(cs[k]) * g[k];
    if (cabs(g[k + 1]) <= gm_rtol * bn) {
      k++;
      status = 0;
      break;
    }
  }
  if (status == 0) {
    /* back substitution H z = g, then y = V z */
    double complex *z = malloc(sizeof(double complex) * k);
    for (int j = k - 1; j >= 0; j--) {
      double complex s = g[j];
      for (int l = j + 1; l < k; l++) s -= Hm[(size_t)j * maxit + l] * z[l];
      z[j] = s / Hm[(size_t)j * maxit + j];
    }
    for (int j = 0; j < k; j++)
      for (int i = 0; i < n; i++) y[i] += z[j] * V[(size_t)n * j + i];
    free(z);
  }
done:
  free(V); free(Hm); free(cs); free(sn); free(g);
  free(re); free(im); free(Lre); free(Lim);
  return status == 0 ? k : -1;
}

int om_rexi_expL(const om_ops *o, double lambda_bar, double t, int N, double eta0,
                 double gm_rtol, double rtol, const double *U, double *out) {
  int n = o->m->ne + o->m->nc;
  double theta = lambda_bar * t;
  double *X = malloc(sizeof(double) * 2 * N), *c = malloc(sizeof(double) * 2 * N);
  double complex *y = malloc(sizeof(double complex) * n);
  double complex *acc = calloc(n, sizeof(double complex));
  om_rexi_coeffs(theta, N, eta0, X, c);
  int status = 0, itmax = 0;
  for (int j = 0; j < N && status == 0; j++) {
    double complex Xj = X[2 * j] + I * X[2 * j + 1];
    double complex cj = c[2 * j] + I * c[2 * j + 1];
    int it = gmres_shifted(o, Xj, lambda_bar, U, y, gm_rtol, rtol, 600);
    if (it < 0) {
      status = -1;
      break;
    }
    if (it > itmax) itmax = it;
    for (int i = 0; i < n; i++) acc[i] += cj * y[i];
  }
  for (int i = 0; i < n; i++) out[i] = creal(acc[i]);
  free(X); free(c); free(y); free(acc);
  return status == 0 ? itmax : -1;
}
