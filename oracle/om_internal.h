/* Oracle internals (TEST INFRASTRUCTURE ONLY, see oracle.h). */
#ifndef OM_INTERNAL_H
#define OM_INTERNAL_H
#include <stdint.h>

struct om_mesh {
  int level;
  double R;
  int nv, ne, nc;
  double *x;   /* nv*3 */
  int *cv;     /* nc*3 vertices, CCW from outside */
  int *ce;     /* nc*3 edge opposite local vertex i */
  int *csign;  /* nc*3 +1 if the edge normal points out of the cell */
  int *ec;     /* ne*2 (c0, c1) */
  int *ev;     /* ne*2 (a, b), CCW around c0 */
};

struct om_ops {
  const struct om_mesh *m;
  double g, H, Omega;
  double *b;      /* nc bottom height (zeros when flat) */
  double *area;   /* nc */
  int nnz;
  int *rowptr;    /* ne+1 */
  int *col;       /* nnz */
  double *mass;   /* nnz: velocity mass matrix */
  double *cor;    /* nnz: Coriolis matrix int f phi_i . (k x phi_j) */
  double *diag;   /* ne: diagonal of the mass matrix */
};

static inline void om_sub(const double *a, const double *b, double *c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
static inline double om_dot(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void om_cross(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Geometry of one flat triangle: vertices p[i], area, unit normal k,
 * orientation signs s[i] and global edges e[i] of the local edges. */
typedef struct {
  double p[3][3];
  double area;
  double k[3];
  int s[3];
  int e[3];
} om_cell;

void om_cell_geom(const struct om_mesh *m, int c, om_cell *T);
/* RT0 basis function i of cell T evaluated at x: s_i (x - p_i) / (2|T|). */
void om_rt0_basis(const om_cell *T, int i, const double *x, double *phi);
/* Velocity of the RT0 field with edge fluxes U on cell T at point x. */
void om_rt0_velocity(const om_cell *T, const double *U, const double *x, double *u);

#endif
