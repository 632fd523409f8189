/*
 * Oracle for the phase-averaged shallow-water right-hand side.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 CPU
 * implementation of what the method computes, written from the paper
 * (Yamazaki, Cotter & Wingate, "Time parallel integration and phase averaging
 * for the nonlinear shallow water equations on the sphere", arXiv 2103.07706).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * Discretisation: lowest-order compatible pair, RT0 velocity fluxes on edges
 * and P0 depth on cells, on an icosahedral mesh of flat triangles whose
 * vertices lie on the sphere (the paper's Sec. 2.5 uses BDM2/P1DG; RT0/P0 is
 * a compatible pair with the same two properties the paper relies on).
 *
 * State vectors are [u (ne edge fluxes, m^2/s) | eta (nc cell values, m)].
 *
 * Parity status per function (what pins it is in tests/test_oracle_*.py):
 *   mesh, operators, mass solve, Chebyshev coefficients and truncation,
 *   exponential, rational exponential, nonlinearity, nodes/weights, averaged
 *   RHS, RK4 step, diagnostics: all pinned.  The velocity upwind direction
 *   inside N is a reading of the paper (its printed inequality selects the
 *   downwind side); the pin of the facet term in closed form (divergence-free
 *   fields, constant per cell) tells the two sides apart.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct om_mesh om_mesh;
typedef struct om_ops om_ops;

/* ---- mesh (Sec. 3, icosahedral grids) ---------------------------------- */
om_mesh *om_mesh_create(int level, double radius);
void om_mesh_destroy(om_mesh *m);
void om_mesh_counts(const om_mesh *m, int *nv, int *ne, int *nc);
/* verts[nv*3]; cell_verts[nc*3] CCW seen from outside; cell_edges[nc*3]
 * (local edge i is opposite local vertex i); cell_sign[nc*3] (+1 when the
 * edge normal points out of the cell); edge_cells[ne*2] (c0<c1, normal out of
 * c0); edge_verts[ne*2] (a->b runs counter-clockwise around c0). Any pointer
 * may be NULL. */
void om_mesh_export(const om_mesh *m, double *verts, int32_t *cell_verts,
                    int32_t *cell_edges, int32_t *cell_sign,
                    int32_t *edge_cells, int32_t *edge_verts);

/* ---- linear operators (Sec. 2.5, discrete L) --------------------------- */
/* b_cell may be NULL (flat bottom). */
om_ops *om_ops_create(const om_mesh *m, double g, double H, double Omega,
                      const double *b_cell);
void om_ops_destroy(om_ops *o);
/* CSR export of the velocity mass matrix and the Coriolis matrix (same
 * pattern): rowptr[ne+1], cols[nnz], mass[nnz], cor[nnz]; area[nc].
 * Returns nnz.  Pass NULL pointers to query nnz only. */
int om_ops_export(const om_ops *o, int32_t *rowptr, int32_t *cols,
                  double *mass, double *cor, double *area);
/* Jacobi-preconditioned CG on M_u x = b from x = 0, stopping when
 * ||r||_2 <= rtol ||b||_2.  Returns the iteration count, -1 on failure. */
int om_mass_solve(const om_ops *o, const double *b, double *x, double rtol,
                  int maxit);
/* out = L U.  Returns 0, or -1 if a mass solve failed. */
int om_apply_L(const om_ops *o, const double *U, double *out, double rtol);
/* Power iteration for rho(L) in the W inner product from start vector v0,
 * 'iters' iterations of v <- L(L v).  Returns the estimate of rho(L). */
double om_power_rho(const om_ops *o, const double *v0, int iters, double rtol);

/* ---- Chebyshev exponential (Sec. 2.4) ---------------------------------- */
/* Chebyshev coefficients a_k (complex, interleaved re/im) of exp(i Lbar x)
 * on [-1,1] by a discrete cosine transform of samples at npts+1 Chebyshev
 * points; a has 2*(npts+1) doubles. */
void om_cheb_coeffs(double Lbar, int npts, double *a);
/* Index of the highest kept coefficient after discarding from the top while
 * the discarded total magnitude stays <= tol. */
int om_cheb_truncate(const double *a, int npts, double tol);
/* out = exp(t L) U by the modified Chebyshev recurrence with
 * Lbar = lambda_bar*|t|.  Returns the degree K used (>=0), -1 on failure. */
int om_expL(const om_ops *o, double lambda_bar, double t, double tol,
            double rtol, const double *U, double *out);

/* ---- rational exponential (REXI, Sec. 2.4 and Sec. 4) ------------------ */
/* Nodes X[N] and coefficients c[N] (complex, interleaved re/im) of the
 * trapezoidal rule of the Cauchy integral of exp(i theta X) over the
 * ellipse X = cosh(eta0 + i phi): r(x) = sum_j c_j / (X_j - x). */
void om_rexi_coeffs(double theta, int N, double eta0, double *X, double *c);
/* out = Re sum_j c_j (X_j I + (i / lambda_bar) L)^{-1} U with theta =
 * lambda_bar t, each shifted system solved by GMRES to gm_rtol (mass solves
 * to rtol).  Returns the largest GMRES iteration count, -1 on failure. */
int om_rexi_expL(const om_ops *o, double lambda_bar, double t, int N, double eta0,
                 double gm_rtol, double rtol, const double *U, double *out);

/* ---- nonlinearity (Sec. 2.5, discrete N) ------------------------------- */
int om_nonlinear(const om_ops *o, const double *U, double *out, double rtol);

/* ---- phase averaging (Sec. 2.2) ---------------------------------------- */
/* Midpoint nodes s[M] on the support of rho(s/T) and normalised weights. */
void om_avg_nodes(int M, double T, double *s, double *w);
/* Nbar = sum_m w_m exp(-s_m L) N(exp(s_m L) U), term by term.
 * which_n selects the inner operator: 0 = SWE nonlinearity, 1 = identity,
 * 2 = the linear operator L (the last two are test hooks). */
int om_phase_avg_rhs(const om_ops *o, double lambda_bar, int nnodes,
                     const double *s, const double *w, double tol,
                     double rtol, int which_n, const double *U, double *out);

/* The same with every exponential the rational (REXI) sum of om_rexi_expL
 * (N nodes, ellipse parameter eta0, GMRES to gm_rtol). */
int om_rexi_phase_avg_rhs(const om_ops *o, double lambda_bar, int nnodes,
                          const double *s, const double *w, int N, double eta0,
                          double gm_rtol, double rtol, int which_n,
                          const double *U, double *out);

/* ---- averaged Lawson RK4 step (Sec. 2.3) ------------------------------- */
/* which_n as for om_phase_avg_rhs. */
int om_step(const om_ops *o, double lambda_bar, int nnodes, const double *s,
            const double *w, double dt, double tol, double rtol, int which_n,
            double *U);
/* The same with every exponential (stages and averages) the REXI sum. */
int om_rexi_step(const om_ops *o, double lambda_bar, int nnodes, const double *s,
                 const double *w, double dt, int N, double eta0, double gm_rtol,
                 double rtol, int which_n, double *U);

/* ---- diagnostics -------------------------------------------------------- */
/* out[0] mass, out[1] linear energy, out[2] nonlinear energy,
 * out[3] H(div) norm of u, out[4] L2 norm of eta. */
void om_diagnostics(const om_ops *o, const double *U, double *out);

#ifdef __cplusplus
}
#endif
#endif
