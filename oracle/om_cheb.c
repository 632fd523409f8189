/*
 * Oracle: the modified-Chebyshev exponential of the paper's Sec. 2.4.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * exp(L t) U is approximated by sum_{k<=N} a_k P_k(L t) U (eq. cheby).  The
 * P_k are Chebyshev polynomials moved from the imaginary interval
 * {iy : |y| <= Lbar} onto [-1, 1], Lbar = |lambda_max| t_max:
 *   P_0 = 1,  P_1(l) = -i l / Lbar,  P_{k+1}(l) = 2 l P_k(l) / (i Lbar) - P_{k-1}(l).
 * The vectors P_k(L t) U are built by that three-term recurrence with one
 * application of L per step.  The a_k are the Chebyshev coefficients of
 * exp(i Lbar x) on [-1, 1] (with x = -i l / Lbar, exp(l) = exp(i Lbar x)),
 * obtained by a discrete cosine transform of samples at Chebyshev points, and
 * coefficients are dropped from the highest degree downwards while the total
 * dropped magnitude stays within the threshold (the paper uses 1e-6).
 *
 * Reading: t_max = |t| for every exponential, so Lbar = lambda_bar |t|
 * (Table 1 counts grow with the time interval, which this reading gives).
 * lambda_bar is an upper estimate of the spectral radius supplied by the
 * caller.  Complex arithmetic is kept exactly as the recurrence is written.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#include "om_internal.h"

void om_cheb_coeffs(double Lbar, int npts, double *a) {
  const double pi = acos(-1.0);
  int N = npts;
  double complex *f = malloc(sizeof(double complex) * (N + 1));
  for (int j = 0; j <= N; j++) f[j] = cexp(I * Lbar * cos(pi * j / N));
  for (int k = 0; k <= N; k++) {
    /* DCT-I: b_k = (2/N) sum'' f_j cos(pi j k / N); halve b_0 and b_N */
    double complex s = 0;
    for (int j = 0; j <= N; j++) {
      double wj = (j == 0 || j == N) ? 0.5 : 1.0;
      s += wj * f[j] * cos(pi * (double)j * (double)k / N);
    }
    s *= 2.0 / N;
    if (k == 0 || k == N) s *= 0.5;
    a[2 * k] = creal(s);
    a[2 * k + 1] = cimag(s);
  }
  free(f);
}

int om_cheb_truncate(const double *a, int npts, double tol) {
  double dropped = 0;
  int K = npts;
  while (K > 0) {
    double mag = hypot(a[2 * K], a[2 * K + 1]);
    if (dropped + mag > tol) break;
    dropped += mag;
    K--;
  }
  return K;
}

/* Number of Chebyshev points used for the coefficients: far enough above
 * Lbar that aliased coefficients are below rounding. */
static int cheb_points(double Lbar) { return 2 * (int)ceil(Lbar) + 64; }

/* Apply L to a complex vector (real and imaginary parts separately). */
static int apply_L_complex(const om_ops *o, const double complex *X,
                           double complex *Y, double rtol) {
  int n = o->m->ne + o->m->nc;
  double *re = malloc(sizeof(double) * n), *im = malloc(sizeof(double) * n);
  double *lre = malloc(sizeof(double) * n), *lim = malloc(sizeof(double) * n);
  for (int i = 0; i < n; i++) {
    re[i] = creal(X[i]);
    im[i] = cimag(X[i]);
  }
  int s1 = om_apply_L(o, re, lre, rtol), s2 = om_apply_L(o, im, lim, rtol);
  for (int i = 0; i < n; i++) Y[i] = lre[i] + I * lim[i];
  free(re); free(im); free(lre); free(lim);
  return (s1 < 0 || s2 < 0) ? -1 : 0;
}

int om_expL(const om_ops *o, double lambda_bar, double t, double tol, double rtol,
            const double *U, double *out) {
  int n = o->m->ne + o->m->nc;
  if (t == 0.0) {
    memcpy(out, U, sizeof(double) * n);
    return 0;
  }
  double Lbar = lambda_bar * fabs(t);
  int N = cheb_points(Lbar);
  double *a = malloc(sizeof(double) * 2 * (N + 1));
  om_cheb_coeffs(Lbar, N, a);
  int K = om_cheb_truncate(a, N, tol);

  double complex *Pm = malloc(sizeof(double complex) * n);  /* P_{k-1} U */
  double complex *P = malloc(sizeof(double complex) * n);   /* P_k U */
  double complex *LP = malloc(sizeof(double complex) * n);
  double complex *acc = malloc(sizeof(double complex) * n);
  int status = 0;
  /* P_0 U = U */
  for (int i = 0; i < n; i++) {
    P[i] = U[i];
    acc[i] = (a[0] + I * a[1]) * P[i];
  }
  for (int k = 0; k < K && status == 0; k++) {
    status = apply_L_complex(o, P, LP, rtol);
    for (int i = 0; i < n; i++) {
      double complex next;
      if (k == 0)
        next = -I * t * LP[i] / Lbar;                   /* P_1 U = -i t L U / Lbar */
      else
        next = 2.0 * t * LP[i] / (I * Lbar) - Pm[i];    /* P_{k+1} U */
      Pm[i] = P[i];
      P[i] = next;
      acc[i] += (a[2 * (k + 1)] + I * a[2 * (k + 1) + 1]) * next;
    }
  }
  /* exp(L t) of a real vector is real; the imaginary part is rounding. */
  for (int i = 0; i < n; i++) out[i] = creal(acc[i]);
  free(a); free(Pm); free(P); free(LP); free(acc);
  return status < 0 ? -1 : K;
}
