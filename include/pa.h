/*
 * pa.h -- C ABI of libpa.so, the MI355X (gfx950) phase-averaged right-hand
 * side of the rotating shallow-water equations.
 *
 * Method: Yamazaki, Cotter & Wingate, "Time parallel integration and phase
 * averaging for the nonlinear shallow water equations on the sphere"
 * (arXiv 2103.07706).  The hot path is the averaged nonlinearity of Sec. 2.2,
 *     Nbar(U) = sum_m w_m exp(-s_m L) N(exp(s_m L) U),
 * with the exponential computed by the modified Chebyshev recurrence of
 * Sec. 2.4 and L, N the compatible finite-element operators of Sec. 2.5 on the
 * lowest-order pair (RT0 edge fluxes, P0 cell depths) of an icosahedral mesh
 * of flat triangles.
 *
 * Conventions
 *  - Every function returns an int status (pa_status); 0 is success.
 *    pa_last_error() returns a thread-local message for the last failure.
 *    No C++ exception crosses this boundary.  Outputs are undefined on error.
 *  - Handles are opaque; each *_create has a matching *_destroy.
 *  - Device memory is owned by the caller: the library reports sizes
 *    (pa_ops_device_size, pa_workspace_size) and works in buffers the caller
 *    binds or passes.  The library itself never allocates device memory.
 *  - Streams are the caller's (a hipStream_t passed as void*); every call
 *    enqueues on the context's stream and synchronises it before returning
 *    (convergence of the mass solves is checked on the host).
 *  - State vectors are FP64 in SI units, one contiguous vector per member:
 *    [u (ne edge fluxes, m^2/s, along the global edge normal) | eta (nc, m)].
 *    A batch of B states is B such vectors back to back.
 *  - "_dev" pointers are device pointers; "_host" pointers are host memory.
 */
#ifndef PA_H
#define PA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PA_OK = 0,
  PA_EINVAL = 1,   /* bad argument or size */
  PA_ENOMEM = 2,   /* caller buffer too small */
  PA_EHIP = 3,     /* HIP runtime error */
  PA_ENOCONV = 4,  /* a mass solve did not reach its tolerance within maxit */
  PA_ENOTSUP = 5,  /* option not supported */
  PA_EGROWTH = 6   /* Chebyshev growth guard tripped (lambda_bar too small) */
} pa_status;

const char *pa_last_error(void);

typedef struct pa_ctx pa_ctx;
typedef struct pa_mesh pa_mesh;
typedef struct pa_ops pa_ops;
typedef struct pa_avg pa_avg;
typedef struct pa_bdm2 pa_bdm2;

/* ---- context -------------------------------------------------------------
 * Binds a device and a stream (hipStream_t, may be NULL for the null stream).
 * Allocates nothing on the device. */
int pa_ctx_create(int device, void *stream, pa_ctx **out);
int pa_ctx_set_stream(pa_ctx *ctx, void *stream);
int pa_ctx_destroy(pa_ctx *ctx);

/* ---- mesh (Sec. 3: icosahedral grids; N_C = 20480 at level 5) ------------
 * Level 0 is the icosahedron; every refinement splits each triangle into four
 * at its edge midpoints, which are moved radially onto the sphere.  Cells are
 * flat triangles, counter-clockwise seen from outside; local edge i is
 * opposite local vertex i; the normal of an edge points out of its
 * lower-numbered cell c0; its endpoints a -> b run counter-clockwise around
 * c0.  level in [0, 9]. */
typedef struct {
  int32_t level, nv, ne, nc;
  double radius;
} pa_mesh_info;
int pa_mesh_icosahedral(int level, double radius, pa_mesh **out);
int pa_mesh_get_info(const pa_mesh *m, pa_mesh_info *info);
/* Host arrays (any may be NULL): verts[nv*3], cell_verts[nc*3],
 * cell_edges[nc*3], edge_cells[ne*2], edge_verts[ne*2]. */
int pa_mesh_export(const pa_mesh *m, double *verts, int32_t *cell_verts,
                   int32_t *cell_edges, int32_t *edge_cells, int32_t *edge_verts);
/* A mesh from the caller's host arrays (copied; same layout as
 * pa_mesh_export): verts[nv*3] on the sphere of the given radius,
 * cell_verts[nc*3], cell_edges[nc*3], edge_cells[ne*2], edge_verts[ne*2].
 * Checked against every convention above (closed, 2 ne = 3 nc; cells
 * counter-clockwise from outside; edge i of a cell joins its vertices
 * i+1 -> i+2; c0 < c1; a -> b counter-clockwise around c0); PA_EINVAL
 * otherwise.  pa_mesh_get_info reports level -1. */
int pa_mesh_from_arrays(int nv, const double *verts, int nc, const int32_t *cell_verts,
                        int ne, const int32_t *cell_edges, const int32_t *edge_cells,
                        const int32_t *edge_verts, double radius, pa_mesh **out);
int pa_mesh_destroy(pa_mesh *m);

/* ---- operators (Sec. 2.5: discrete L and N) ------------------------------
 * Host assembly of the velocity mass matrix, the Coriolis matrix
 * (f = 2 Omega sin(latitude) at the cell quadrature points), the divergence
 * and the cell areas, plus the per-cell/per-edge geometry N needs (the
 * nonlinear cell term as per-cell forms in the cell's edge fluxes).
 * b_cell (nc values, may be NULL) is the bottom height.  lambda_bar is the
 * Chebyshev scale |lambda_max| of Sec. 2.4 (an upper estimate of the spectral
 * radius of L); 0 means "estimate it" (pa_ops_estimate_lambda). */
typedef struct {
  double g, H, omega;
  const double *b_cell;
  double lambda_bar;
} pa_phys;
int pa_ops_create(const pa_mesh *m, const pa_phys *phys, pa_ops **out);
/* Bytes of device memory the operators occupy. */
int pa_ops_device_size(const pa_ops *ops, size_t *bytes);
/* Upload the operators into the caller's device buffer (>= device_size
 * bytes, 256-byte aligned).  The buffer must outlive the ops and must not
 * be written by the caller while work of calls on the ops is in flight
 * (kernels read its tables through the scalar data cache). */
int pa_ops_bind(pa_ctx *ctx, pa_ops *ops, void *dev_buf);
/* Power iteration on the GPU, v <- L(L v) in the energy inner product, from
 * a fixed start vector; sets lambda_bar = safety * estimate of rho(L).
 * Needs a workspace of pa_workspace_size(ops, NULL, 1, cfg). */
int pa_ops_estimate_lambda(pa_ctx *ctx, pa_ops *ops, int iters, double safety,
                           void *ws_dev, size_t ws_bytes, double *lambda_bar);
int pa_ops_set_lambda(pa_ops *ops, double lambda_bar);
int pa_ops_get_lambda(const pa_ops *ops, double *lambda_bar);
int pa_ops_destroy(pa_ops *ops);

/* ---- averaging (Sec. 2.2) ------------------------------------------------
 * M midpoint nodes on the support of rho(s/T): s_m = T(-1/2 + (m+1/2)/M),
 * weights w_m = rho(s_m/T) / sum_j rho(s_j/T), rho(x) = exp(-1/(1/4 - x^2)).
 * (Readings: the printed weight's exponent has the wrong sign; the weights
 * are normalised discretely; the nodes cover the support |s| < T/2.)
 * pa_avg_create_nodes takes explicit nodes and weights instead. */
int pa_avg_create(int M, double T, pa_avg **out);
int pa_avg_create_nodes(int M, const double *s_host, const double *w_host,
                        pa_avg **out);
int pa_avg_nodes(const pa_avg *avg, double *s_host, double *w_host);
int pa_avg_destroy(pa_avg *avg);

/* ---- solve configuration -------------------------------------------------- */
enum { PA_FP64 = 0, PA_FP32_REFINED = 1 };
enum { PA_BACKWARD_PER_TERM = 0, PA_BACKWARD_CLENSHAW = 1 };
typedef struct {
  int32_t precision;   /* PA_FP64, or PA_FP32_REFINED: mass solves on column
                          blocks at least mixed_min_cols wide (launch shape,
                          below) run FP32 Chebyshev inner solves (FP32 copy
                          of M_u, to max(inner_rtol, 1e-6)) inside FP64
                          refinement (x += x32, r -= M x32 with the FP64
                          matrix), narrower ones FP64 Chebyshev steps; the
                          final FP64 residual is checked against cg_rtol and
                          a failed check repeats the call in FP64.  The
                          recurrences, stiffness, N and all sums stay FP64. */
  int32_t backward;    /* how the M backward exponentials are summed */
  int32_t maxit;       /* CG iterations per mass solve (FP64) */
  int32_t growth_guard;/* 1: after the forward Chebyshev basis of each averaged
                          right-hand side (up to four per call), compare the
                          energy norm of the last basis vector with that of
                          the state (never larger when lambda_bar >= rho(L),
                          Sec. 2.4); growth above 1% fails the call with
                          PA_EGROWTH, stats.guard_trips counting the states */
  double cg_rtol;      /* ||r||_2 <= cg_rtol ||b||_2 for every mass solve */
  double cheb_tol;     /* Chebyshev truncation threshold (paper: 1e-6) */
  double weight_cut;   /* skip terms with w_m < weight_cut * max_j w_j */
  double inner_rtol;   /* FP32 inner solve tolerance (PA_FP32_REFINED) */
  int32_t use_graph;   /* 1: capture pa_phase_avg_rhs into a HIP graph once an
                          iteration budget is known and replay it while its
                          inputs (pointers, sizes, settings) stay the same */
  int32_t solver;      /* mass solves: PA_SOLVER_CG (Jacobi-preconditioned
                          CG, as in the paper's method) or PA_SOLVER_CHEBYSHEV
                          (Jacobi-preconditioned Chebyshev semi-iteration over
                          Lanczos bounds of the spectrum of D^-1 M: no inner
                          products, step count fixed by the bounds, final FP64
                          residual checked against cg_rtol; a failed check
                          repeats the call with CG) */
  int32_t precond;     /* PA_PRECOND_JACOBI, or PA_PRECOND_LEARNED: the
                          Chebyshev mass solves (solver PA_SOLVER_CHEBYSHEV,
                          precision PA_FP64) may use the learned P = G G^T
                          bound to the operators (pa_ops_lp_attach +
                          pa_ops_lp_bind; PA_EINVAL if none is bound), with
                          steps from the Ritz bounds of P M.  Each solve
                          takes the learned or the Jacobi steps, whichever
                          moves fewer bytes: steps x (48 bytes per row and
                          column for x, r, d in and out, plus the matrix rows
                          of one launch: 68 bytes for Jacobi, 60 + 8 (w_P +
                          w_PM) learned), so learned for wide column blocks.
                          The final FP64 residual check and its CG repeat
                          are as for Jacobi.  CG and FP32-refined solves use
                          Jacobi. */
  int32_t exponential; /* PA_EXP_CHEBYSHEV: the Chebyshev polynomial of
                          Sec. 2.4 (above).  PA_EXP_REXI: the rational sum
                          that Sec. 2.4 and Sec. 4 name as the parallel
                          alternative, every exponential of the call (those
                          of the average, the stages of pa_step) as
                            exp(t L) U ~ Re sum_{j<N} c_j (X_j + (i/lb) L)^-1 U,
                            X_j = cosh(eta0 + i phi_j), phi_j = 2 pi (j+1/2)/N,
                            c_j = exp(i theta X_j) sinh(eta0 + i phi_j) / N,
                          theta = lb t, lb = lambda_bar: the N-point
                          trapezoidal rule of the Cauchy integral of
                          exp(i theta x) over the ellipse with foci -1, 1
                          through X_0 (Trefethen and Weideman, SIAM Review
                          56, 2014).  The nodes pair up as X and -conj(X)
                          with conjugate terms, so N/2 complex solves carry
                          the sum.  The poles do not depend on t: the M
                          forward exponentials of the average share the N/2
                          solves of U, and the weighted backward sum is N/2
                          solves of complex combinations of the N(E_m).
                          Each shifted system is solved through its velocity
                          Schur complement
                            (X M_u - (i/lb) F - gH/(lb^2 X) D' A^-1 D) y_u
                              = M_u U_u - i g/(lb X) D' U_eta,
                            y_eta = (U_eta + i H/lb A^-1 D y_u) / X
                          (A the cell areas), by Jacobi-preconditioned
                          BiCGStab with the true residual checked against
                          cg_rtol (a failed check restarts from the iterate,
                          maxit iterations at most).  precision, solver,
                          precond, backward and use_graph then concern the
                          mass solves of N only, and calls do not capture
                          graphs (convergence is polled). */
  int32_t rexi_nodes;  /* PA_EXP_REXI: N, a multiple of 4 in [8, 256], with
                          rexi_eta0 in (0, 3]; 0: the library takes the pair
                          of smallest N / eta0 (the solves' iteration count
                          grows like 1/eta0) whose rational function is
                          within cheb_tol / 2 of exp(i theta x) on [-1, 1] at
                          the largest theta of the call and whose solve
                          error, sum_j |c_j| / dist(X_j, [-1, 1]) cg_rtol,
                          stays below cheb_tol / 2 */
  double rexi_eta0;
} pa_solve_cfg;
enum { PA_EXP_CHEBYSHEV = 0, PA_EXP_REXI = 1 };
enum { PA_PRECOND_JACOBI = 0, PA_PRECOND_LEARNED = 1 };
enum { PA_SOLVER_CG = 0, PA_SOLVER_CHEBYSHEV = 1 };
/* Defaults: the fastest FP64 form measured on MI355X at the throughput
 * workload -- PA_FP64, PA_BACKWARD_CLENSHAW, PA_SOLVER_CHEBYSHEV,
 * PA_PRECOND_JACOBI, use_graph 1, maxit 100, cg_rtol 1e-10, cheb_tol 1e-6
 * (the paper's threshold), weight_cut 1e-16, inner_rtol 1e-6, growth_guard
 * 0.  (PA_FP32_REFINED is faster still on wide column blocks; it is a
 * precision choice left to the caller.)  pa_step always solves with FP64
 * CG: it works in place, so a failed check could not be repeated. */
void pa_solve_cfg_default(pa_solve_cfg *cfg);

/* Statistics of the last call (valid when the call returns). */
typedef struct {
  int32_t solves;        /* batched mass solves issued */
  int32_t cg_iters;      /* CG iterations summed over solves (batch max each) */
  int32_t cg_iters_max;  /* largest iteration count of one solve */
  int32_t kmax;          /* largest Chebyshev degree used */
  int32_t ksum;          /* sum of per-term degrees (backward) */
  int32_t terms;         /* averaging terms evaluated */
  int32_t refinements;   /* FP64 refinement sweeps (PA_FP32_REFINED) */
  int32_t guard_trips;
  double resid_max;      /* largest final relative residual of a Chebyshev
                            mass solve (its true residual, checked); CG
                            solves stop on their own recursive residual and
                            leave it 0 */
  double device_ms;      /* device time of the call */
  int32_t graph;         /* 1 if the call ran as a graph replay or capture */
  int32_t budget;        /* CG iterations per solve launched (0: polled) */
  int32_t precond;       /* PA_PRECOND_LEARNED if any solve used it */
  int32_t lp_solves;     /* mass solves that used the learned preconditioner */
  int32_t fallbacks;     /* repeats of the call: a CG budget overrun (with
                            polling) or a failed Chebyshev check (with FP64
                            CG); the other fields describe the last run */
  int32_t graph_captured;/* 1 if this call captured a new graph: the first
                            graph call, or one after anything the graph
                            depends on changed (pointers, sizes, settings,
                            launch shape, operator contents or buffers,
                            averaging nodes) */
  int32_t rexi_nodes;    /* PA_EXP_REXI: N of the call's rational sums */
  int32_t rexi_solves;   /* PA_EXP_REXI: batched shifted solves issued */
  int32_t rexi_iters;    /* BiCGStab iterations summed over those solves
                            (the batch's count each) */
  int32_t rexi_iters_max;/* largest iteration count of one column */
  int32_t rexi_restarts; /* restarts after a failed true-residual check */
  int32_t rexi_pad;
  double rexi_eta0;      /* ellipse parameter of the call's rational sums */
  double rexi_resid_max; /* largest final true relative residual of a
                            shifted solve */
} pa_stats;

/* Device workspace bytes for calls on 'batch' states (expL_apply,
 * swe_nonlinear: batch = B; phase_avg_rhs, step: batch = members, avg given).
 * Pass avg = NULL for calls that do not average.  With PA_EXP_REXI the
 * node count of the rational sum, and so the workspace, grows with
 * lambda_bar |t|: for expL_apply the size covers the largest node count
 * (256) unless cfg->rexi_nodes fixes it, and for pa_step it covers dt up to
 * max |s_m| (a call that needs more fails with PA_ENOMEM). */
int pa_workspace_size(const pa_ops *ops, const pa_avg *avg, int batch,
                      const pa_solve_cfg *cfg, size_t *bytes);

/* exp(t_j L) U_j for j < B (Sec. 2.4): the modified Chebyshev recurrence
 * with Lbar = lambda_bar |t_j|, truncated at cfg->cheb_tol; every
 * application of L solves the velocity mass matrix by Jacobi-preconditioned
 * CG.  U_in_dev, U_out_dev: B state vectors (may alias). */
int pa_expL_apply(pa_ctx *ctx, const pa_ops *ops, int B, const double *t_host,
                  const double *U_in_dev, double *U_out_dev, void *ws_dev,
                  size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats);

/* N(U_j) for j < B (Sec. 2.5, discrete nonlinear operator; upwind value from
 * the cell the edge flux leaves, facet value of eta - b upwind). */
int pa_swe_nonlinear(pa_ctx *ctx, const pa_ops *ops, int B, const double *U_dev,
                     double *NU_dev, void *ws_dev, size_t ws_bytes,
                     const pa_solve_cfg *cfg, pa_stats *stats);

/* Nbar(U_j) for each of 'members' states (Sec. 2.2, eq. vt_discretised):
 * forward exponentials from one shared Chebyshev basis, N on all M shifted
 * states, backward exponentials summed with the weights. */
int pa_phase_avg_rhs(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg,
                     int members, const double *U_dev, double *Nbar_dev,
                     void *ws_dev, size_t ws_bytes, const pa_solve_cfg *cfg,
                     pa_stats *stats);

/* pa_phase_avg_rhs without a workspace argument, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a static device array
 * of 256 MiB inside the library (each GPU the library runs on holds its own
 * copy until the process ends; its address is looked up once per device);
 * the call allocates no device memory and captures no graph (cfg->use_graph
 * is ignored: instantiating a graph allocates).  A problem whose workspace
 * (pa_workspace_size, for cfg and for the FP64 CG repeat) exceeds 256 MiB
 * fails with PA_ENOMEM before anything is launched: one member at level 4
 * with M = 64 fits, one member at level 5 with M = 32 in FP64 fits, level 6
 * does not.  The scratch keeps the last call's contents; every call clears
 * what must start at zero.  Calls on one GPU share the scratch, so calls that
 * overlap on one GPU (two threads, two streams) race: serialise them.
 * Arguments, results and errors otherwise as pa_phase_avg_rhs. */
int pa_phase_avg_rhs_noalloc(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg,
                             int members, const double *U_dev, double *Nbar_dev,
                             const pa_solve_cfg *cfg, pa_stats *stats);

/* One step of the averaged Lawson RK4 scheme (Sec. 2.3, four stages), in
 * place on 'members' states. */
int pa_step(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, double dt,
            int members, double *U_dev_inout, void *ws_dev, size_t ws_bytes,
            const pa_solve_cfg *cfg, pa_stats *stats);

/* FP64 diagnostics of B states into out_host[B*5]: mass sum |c| eta,
 * linear energy (H u'M u + g sum |c| eta^2)/2, nonlinear energy
 * sum_c (H + eta - b) int |u|^2/2 + g |c| eta^2 / 2, H(div) norm of u,
 * L2 norm of eta. */
int pa_diagnostics(pa_ctx *ctx, const pa_ops *ops, int B, const double *U_dev,
                   void *ws_dev, size_t ws_bytes, double *out_host);

/* ---- measurement hook -----------------------------------------------------
 * Brackets the launches of one kernel on the context's stream with HIP
 * events (one pair around the back-to-back launches of each mass solve) and
 * counts the algorithmic bytes they move (operands each launch must stream
 * at least once, for the columns still active in it).  Kernels:
 *   PA_KERNEL_CG_ITER      CG iteration (k_cg_iter)
 *   PA_KERNEL_CHEB_ITER    two-term Jacobi Chebyshev step (k_cheb_iter)
 *   PA_KERNEL_CHEB_LP_ITER learned-preconditioner step (k_cheb_lp_iter; the
 *                          two-kernel wide form counts both kernels)
 *   PA_KERNEL_CHEB_FUSED   fused single-column steps (k_cheb_fused)
 *   PA_KERNEL_CHEB3_ITER   three-term block step (k_cheb3_iter)
 *   PA_KERNEL_CHEB32_ITER  FP32 three-term step (k_cheb32_iter[4])
 *   PA_KERNEL_B2_STEP      BDM2 mass-solve step, three-term form (k_b2_step3,
 *                          row form: per row the ELL row's 21 values, a third
 *                          of its block's 7 column-block ids and D^-1, 185.3
 *                          bytes; element form on 8 to 32 columns, k_b2_mel
 *                          + k_b2_step3_el, and cell form on 64, k_b2_cstep:
 *                          per cell its 12 x 12 block, per row D^-1; per row
 *                          and column 32 bytes in all three; FP64 steps
 *                          only, not the FP32 inner steps of
 *                          PA_FP32_REFINED solves)
 * pa_ctx_profile starts a new tally (PA_KERNEL_NONE switches it off and
 * graph capture is not used while it is on); pa_ctx_profile_read returns the
 * tally so far.  The calls made while the hook is on fill it; reading needs
 * no further synchronisation. */
enum { PA_KERNEL_NONE = 0, PA_KERNEL_CG_ITER = 1, PA_KERNEL_CHEB_ITER = 2,
       PA_KERNEL_CHEB_LP_ITER = 3, PA_KERNEL_CHEB_FUSED = 4, PA_KERNEL_CHEB3_ITER = 5,
       PA_KERNEL_CHEB32_ITER = 6, PA_KERNEL_B2_STEP = 7 };
typedef struct {
  int64_t launches;   /* launches of the kernel */
  int64_t work_launches; /* launches that found active columns */
  double total_ms;    /* summed event time of all launches */
  double bytes;       /* algorithmic bytes of all launches */
  double units;       /* mass-solve steps (iterations) times the columns they
                         ran on, summed over the launches */
} pa_kernel_profile;
int pa_ctx_profile(pa_ctx *ctx, int kernel);
/* Iteration budget of the mass solves.  After a call whose outputs do not
 * alias its inputs, the context remembers (per cg_rtol) the largest CG
 * iteration count plus two; later such calls launch exactly that many
 * iterations with no host polling and check convergence once at the end,
 * repeating the call with polling if a column outlived the budget.  This
 * sets (iters > 0) or clears (iters = 0) the remembered value, e.g. to test
 * the repeat path. */
int pa_ctx_set_cg_budget(pa_ctx *ctx, double cg_rtol, int iters);

/* ---- launch shape and autotuner -------------------------------------------
 * Row-parallel kernels take their grid from a launch shape: rows per thread
 * for batches of at most 4 columns (latency-bound), and the workgroup cap
 * per column tile for wider batches.  lp_min_cols is the narrowest column
 * block whose mass solves take learned steps when the learned
 * preconditioner is enabled (narrower blocks take Jacobi steps; a learned
 * step costs more than a Jacobi step, so fewer steps pay only on wide
 * enough blocks).  mixed_min_cols likewise is the narrowest block whose
 * mass solves run as FP32 solves with FP64 refinement when cfg asks for
 * PA_FP32_REFINED (narrower blocks take FP64 steps, which are launch bound
 * there; the FP64 residual check is the same).  fused_steps (1 to 6) is the
 * number of Jacobi Chebyshev steps of a single-column mass solve per launch
 * (a workgroup owns a part of 512 rows and forms the earlier steps again on
 * the rings of rows its later steps read; the results are the same as one
 * step per launch).
 *
 * Which shape a call uses: a batch item's own shape (pa_batch_set_tune),
 * else the operators' own shape (pa_ops_set_tune, pa_autotune), else the
 * process default (pa_get/set_launch_tune, guarded by a lock).  A call reads
 * its shape once when it starts, so calls on different operators from
 * different threads do not affect each other's shapes.
 *
 * pa_autotune times pa_phase_avg_rhs over a small set of shapes on the
 * given problem (the workspace must fit it), then, with the learned
 * preconditioner or FP32 refinement enabled in cfg, over lp_min_cols and
 * mixed_min_cols in {1, 8, 64, never}, then over fused_steps, then over the
 * shapes once more with the fields found, and stores the fastest as the
 * operators' own shape (the process default is left as it is); it returns
 * the choice and the best time.  pa_ops_set_tune with t = NULL drops the
 * operators' own shape; pa_ops_get_tune returns the shape the operators'
 * calls use and (own, may be NULL) whether it is their own. */
typedef struct {
  int32_t narrow_rows_per_thread;
  int32_t wide_max_wg;
  double best_ms;
  int32_t lp_min_cols;
  int32_t mixed_min_cols;
  int32_t fused_steps;
} pa_launch_tune;
int pa_get_launch_tune(pa_launch_tune *out);
int pa_set_launch_tune(const pa_launch_tune *t);
int pa_ops_set_tune(pa_ops *ops, const pa_launch_tune *t);
int pa_ops_get_tune(const pa_ops *ops, pa_launch_tune *out, int *own);
int pa_autotune(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg, int members,
                const double *U_dev, double *out_dev, void *ws_dev,
                size_t ws_bytes, const pa_solve_cfg *cfg, pa_launch_tune *out);
int pa_ctx_profile_read(pa_ctx *ctx, pa_kernel_profile *out);


/* ---- learned mass-matrix preconditioner -----------------------------------
 * The paper solves the velocity mass systems by preconditioned conjugate
 * gradients (end of Sec. 2.5); this preconditioner is an addition to it.  A
 * message-passing network on the edge-cell graph of the mesh maps local
 * geometry to a sparse factor Ghat with the mass-matrix pattern; the
 * preconditioner is P = D^-1/2 Ghat Ghat^T D^-1/2 (D = diag M_u), symmetric
 * positive definite whenever Ghat is non-singular.
 *
 * Network (width 32, relu):
 *   edge features (8): M_ee; |e| / mean edge length; (|c0| + |c1|) / (2 mean
 *     area); z/|x| at the midpoint; mean and |difference| of the cosines of
 *     the two angles opposite e; mean and (max - min) of the four cosines of
 *     the angles at the endpoints of e;
 *   cell features (4): |c| / mean area; z/|x| at the centroid; max - min of
 *     the cosines of its angles; mean M_ee over its edges;
 *   he = relu(Fe W_ee + b_ee), hc = relu(Fc W_ce + b_ce); three rounds of
 *     hc = relu([hc, mean he over the cell's edges] W_cl + b_cl),
 *     he = relu([he, mean hc over the edge's cells] W_el + b_el);
 *   Ghat_ii = softplus(he_i . w_hd + b_hd); for distinct edges i, j of a
 *     cell c: Ghat_ij = (relu([he_i, he_j, hc_c] W_p1 + b_p1) . w_p2 + b_p2)
 *     * M_ij / sqrt(M_ii M_jj).
 * Parameters (16098 floats) in storage order W_ee [8][32], b_ee, W_ce
 * [4][32], b_ce, then per round W_cl [64][32], b_cl, W_el [64][32], b_el,
 * then w_hd [32], b_hd, W_p1 [96][32], b_p1, w_p2 [32], b_p2.  Initial
 * values: Glorot-uniform weights from SplitMix64(seed), zero biases and
 * head weights, b_hd = log(e - 1): Ghat = I, i.e. Jacobi.
 * Loss over probe vectors z_p: (1/P) sum_p |Ghat^T Mhat Ghat z_p - z_p|^2 /
 * |z_p|^2 with Mhat = D^-1/2 M_u D^-1/2 (zero iff P M_u = I).
 * Dense layers run on the matrix cores: BF16 inputs and weights with FP32
 * accumulation (bf16 = 1) or FP32 (bf16 = 0); the loss and the heads in
 * FP64.  Network state is a host object; every call uploads what it needs. */
typedef struct pa_lp pa_lp;
int pa_lp_create(int layers, int width, uint64_t seed, pa_lp **out); /* 3, 32 only */
int pa_lp_param_count(const pa_lp *lp, int *n);
int pa_lp_get_params(const pa_lp *lp, float *out);
int pa_lp_set_params(pa_lp *lp, const float *in);
int pa_lp_save(const pa_lp *lp, const char *path);   /* raw little-endian file */
int pa_lp_load(pa_lp *lp, const char *path);
int pa_lp_destroy(pa_lp *lp);

typedef struct {
  int32_t steps;     /* Adam steps; each takes one Rademacher probe block per operator */
  int32_t probes;    /* probe vectors per block, 1..16 */
  double lr;         /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
  int32_t bf16;      /* 1: BF16 matrix-core layers, 0: FP32 */
  uint64_t seed;     /* probe seed */
} pa_train_cfg;
typedef struct {
  double loss_first, loss_last;  /* mean loss over operators, first and last step */
  double ms;                     /* wall time of the call */
  int32_t steps;
} pa_train_stats;
/* Device workspace for training on (or evaluating) the given operators. */
int pa_lp_workspace_size(const pa_ops *const *ops, int n_ops, int probes, int steps,
                         size_t *bytes);
/* Trains lp in place on the GPU: every step sums the loss gradient over the
 * operators (fresh probes each) and applies one Adam update. */
int pa_lp_train(pa_ctx *ctx, pa_lp *lp, const pa_ops *const *ops, int n_ops,
                const pa_train_cfg *cfg, void *ws_dev, size_t ws_bytes,
                pa_train_stats *stats);
/* Test hooks: the loss and its gradient (n_params doubles) for probes given
 * on the host as [n_e][n_probe]; and Ghat (diagonal [n_e], off-diagonal
 * [n_e][4] in the operator's mass-pattern slot order: the other two edges
 * of the edge's first cell, then of its second cell). */
int pa_lp_loss_grad(pa_ctx *ctx, const pa_lp *lp, const pa_ops *ops, int n_probe,
                    const double *probes_host, int bf16, void *ws_dev, size_t ws_bytes,
                    double *loss, double *grad_host);
int pa_lp_ghat(pa_ctx *ctx, const pa_lp *lp, const pa_ops *ops, int bf16, void *ws_dev,
               size_t ws_bytes, double *gdiag_host, double *goff_host);

/* Attaching: inference on the operator's graph, then on the host P and P M
 * as ELL tables (FP32 values) and the Ritz bounds of P M (Lanczos).  The
 * tables are then bound to caller-owned device memory like the operators. */
typedef struct {
  double eig_min, eig_max;                /* Ritz bounds of P M */
  double jacobi_eig_min, jacobi_eig_max;  /* Ritz bounds of D^-1 M */
  int32_t width_p, width_pm;              /* ELL widths of P and P M */
} pa_lp_info;
int pa_ops_lp_attach(pa_ctx *ctx, pa_ops *ops, const pa_lp *lp, int bf16, void *ws_dev,
                     size_t ws_bytes, pa_lp_info *info);
int pa_ops_lp_device_size(const pa_ops *ops, size_t *bytes);
int pa_ops_lp_bind(pa_ctx *ctx, pa_ops *ops, void *dev_buf);

/* ---- batches of problems -------------------------------------------------
 * Independent problems evaluated together (the terms of the average are
 * independent, Sec. 2.2, and were spread over an ensemble of processes,
 * end of Sec. 2.5; members and meshes are independent too): a batch holds
 * n_items averaged right-hand-side problems, item i being `members[i]`
 * states on the operators `ops[i]` (meshes may differ), all with the same
 * averaging nodes `avg`.  pa_batch_run evaluates Nbar for every item:
 * U_dev[i] and Nbar_dev[i] are FP64 device arrays [members[i]][n_i] as in
 * pa_phase_avg_rhs.
 *
 * Execution: when no mass solve needs host polling (Chebyshev or mixed
 * precision solver, or a learned CG budget), the items run concurrently on
 * streams owned by the batch, joined back into the context stream; with
 * cfg->use_graph the whole batch is captured on the first run into one HIP
 * graph and replayed on later runs with the same pointers, configuration,
 * operators and launch shapes (any change recaptures).  Otherwise the items
 * run one after another on the context stream.  Each item uses its own
 * launch shape (pa_batch_set_tune / pa_batch_autotune), default the
 * process-wide one.
 *
 * Workspace: pa_batch_workspace_size gives the bytes for `cfg`, the items
 * carved one after another (256-byte aligned).  The batch does not own the
 * operators or the averaging nodes, which must outlive it.  `stats` (may be
 * NULL) receives n_items entries.  Errors as pa_phase_avg_rhs; calls on one
 * batch are not thread-safe. */
typedef struct pa_batch pa_batch;
int pa_batch_create(int n_items, const pa_ops *const *ops, const int *members,
                    const pa_avg *avg, pa_batch **out);
int pa_batch_workspace_size(const pa_batch *b, const pa_solve_cfg *cfg, size_t *bytes);
int pa_batch_run(pa_ctx *ctx, pa_batch *b, const double *const *U_dev,
                 double *const *Nbar_dev, void *ws_dev, size_t ws_bytes,
                 const pa_solve_cfg *cfg, pa_stats *stats);
/* Launch shape of one item (best_ms ignored). */
int pa_batch_set_tune(pa_batch *b, int item, const pa_launch_tune *t);
int pa_batch_get_tune(const pa_batch *b, int item, pa_launch_tune *out);
/* Times each item alone over the launch shapes of pa_autotune (outputs must
 * not alias inputs) and keeps each item's fastest; out (may be NULL)
 * receives n_items entries.  The process-wide shape is left unchanged. */
int pa_batch_autotune(pa_ctx *ctx, pa_batch *b, const double *const *U_dev,
                      double *const *Nbar_dev, void *ws_dev, size_t ws_bytes,
                      const pa_solve_cfg *cfg, pa_launch_tune *out);
int pa_batch_destroy(pa_batch *b);

/* ---- the paper's own spaces: BDM2 velocity x P1DG depth (Sec. 2.5) -------
 * The linear operator of eq. ueq_int and the depth equation after it,
 *   L(u, eta) = (M_u^-1 (-F u + g B eta), M_h^-1 (-H B^T u)),
 * M_u[i,j] = int phi_i . phi_j, F[i,j] = int phi_i . (f k x phi_j)
 * (f = 2 omega z/|x| at the quadrature points), B[i,q] = int div(phi_i) psi_q,
 * M_h[q,r] = int psi_q psi_r, on the flat cells of a mesh, and exp(t L) U by
 * the Chebyshev polynomial of Sec. 2.4 on it.  Unknowns of a state (length
 * nu + nh, velocity first):
 *   3 e + k      the normal component of u at Gauss-Legendre point k of edge
 *                e (points from the edge's a to its b; the normal in the
 *                plane of cell c0, pointing out of c0),
 *   3 ne + 3 c + m  the interior moments of cell c: the integrals of u . e1
 *                and u . e2 over the cell divided by its area A, and of
 *                u . (x - x_c)^perp divided by A^1.5 (e1 = unit vector from
 *                the cell's vertex 0 to vertex 1, e2 = k x e1, x_c the
 *                centroid, perp a quarter turn about k),
 *   nu + 3 c + q the coefficient of the barycentric coordinate of the
 *                cell's vertex q in the depth.
 * nu = 3 ne + 3 nc, nh = 3 nc.  Integrals: collapsed Gauss-Legendre rule of
 * 5 x 5 points per cell.  The mass solves M_u^-1 are Jacobi Chebyshev
 * semi-iterations over the Ritz bounds of D^-1 M_u (widened 3% below and 1%
 * above) to cg_rtol, checked in FP64 (PA_ENOCONV if a check fails); M_h^-1
 * is exact (block diagonal).  phys->b_cell must be NULL (the bottom of this
 * pair is P1DG: pa_bdm2_set_bottom); lambda_bar is the
 * scale of the Chebyshev polynomial (set it, e.g. to rho(L) times a safety
 * factor, before an exponential). */
int pa_bdm2_create(const pa_mesh *m, const pa_phys *phys, pa_bdm2 **out);
/* nu, nh, and the Ritz bounds of D^-1 M_u (any pointer may be NULL). */
int pa_bdm2_info(const pa_bdm2 *b, int32_t *nu, int32_t *nh, double *eig_min,
                 double *eig_max);
/* Host copies of the assembled tables (any pointer may be NULL), rows
 * column-major so that entry s of row i sits at s * nu + i:
 * col, mass, cor [21 * nu] (the columns of M_u and F, unused slots point at
 * the row itself with value 0), bcol, bval [6 * nu] (B; unused slots
 * column 0, value 0), cdof [nc * 12] (velocity unknowns of each cell: its
 * edges' 3 points each, edge i of the cell first, then its 3 moments), and
 * q [nc * 3 * 12] (-H M_h^-1 B^T restricted to the cell, so that depth row
 * 3 c + r of L u is sum_k q[(3 c + r) * 12 + k] u[cdof[12 c + k]]). */
int pa_bdm2_tables(const pa_bdm2 *b, int32_t *col, double *mass, double *cor,
                   int32_t *bcol, double *bval, int32_t *cdof, double *q);
/* Device bytes of the tables; bind uploads them into the caller's buffer
 * (256-byte aligned, kept alive and unwritten while calls run). */
int pa_bdm2_device_size(const pa_bdm2 *b, size_t *bytes);
int pa_bdm2_bind(pa_ctx *ctx, pa_bdm2 *b, void *dev_buf);
/* Bottom height b as P1DG coefficients (nh host values, copied; NULL: flat),
 * before pa_bdm2_bind (PA_EINVAL after).  Only N sees it: its depth flux
 * carries eta - b (L keeps the mean depth H). */
int pa_bdm2_set_bottom(pa_bdm2 *b, const double *bottom_host);
int pa_bdm2_set_lambda(pa_bdm2 *b, double lambda_bar);
/* Power iteration on the GPU, v <- -L^2 v normalised in the energy norm
 * H u' M_u u + g eta' M_h eta (L is skew in it), from a fixed start vector
 * (a counter hash of the index); sets lambda_bar = safety * the estimate of
 * rho(L), which approaches rho(L) from below.  Mass solves to 1e-12.
 * Needs a workspace of pa_bdm2_workspace_size(b, PA_BDM2_APPLY_L, 1, ...). */
int pa_bdm2_estimate_lambda(pa_ctx *ctx, pa_bdm2 *b, int iters, double safety,
                            void *ws_dev, size_t ws_bytes, double *lambda_bar);
/* Workspace bytes of a call: call is one of the PA_BDM2_* values below, B
 * the number of states (members for PA_BDM2_PHASE_AVG); t_host the B times
 * of PA_BDM2_EXPL (the degree depends on them), avg the nodes of
 * PA_BDM2_PHASE_AVG (others NULL).  B < 1 is PA_EINVAL; L, the exponential
 * and N take at most 64 states (PA_ENOTSUP beyond), the step at most 64
 * members (PA_EINVAL beyond), the average any number. */
enum { PA_BDM2_APPLY_L = 0, PA_BDM2_EXPL = 1, PA_BDM2_NONLINEAR = 2, PA_BDM2_PHASE_AVG = 3,
       PA_BDM2_STEP = 4 };  /* PA_BDM2_STEP: t_host points to dt */
int pa_bdm2_workspace_size(const pa_bdm2 *b, int call, int B, const double *t_host,
                           const pa_avg *avg, const pa_solve_cfg *cfg, size_t *bytes);
/* out = L U for B states, member-major [B][nu + nh] in device memory (out
 * must not alias U).  cfg: cg_rtol and maxit (the cap on semi-iteration
 * steps) apply, and cheb_tol, weight_cut and backward where the call has an
 * exponential or an average; NULL takes the defaults.  The pair's solves
 * are Jacobi Chebyshev semi-iterations and its exponential is the
 * Chebyshev one.  With precision PA_FP32_REFINED the solves on 64-column
 * blocks run FP32 inner rounds to max(inner_rtol, 1e-6) closed by FP64
 * refinements of x and r (narrower blocks stay FP64); the FP64 residual
 * check decides either way.  A cfg asking for PA_EXP_REXI, PA_SOLVER_CG or
 * PA_PRECOND_LEARNED is refused with PA_ENOTSUP (use_graph is ignored).
 * Every call's workspace is 256-byte aligned (PA_EINVAL).  stats (may be
 * NULL): solves, cg_iters (steps summed, inner FP32 steps included),
 * cg_iters_max, refinements, resid_max, device_ms. */
int pa_bdm2_apply_L(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *U_dev,
                    double *out_dev, void *ws_dev, size_t ws_bytes,
                    const pa_solve_cfg *cfg, pa_stats *stats);
/* U_out[j] = exp(t_j L) U_in[j] for B states by sum_k c_k R_k:
 * R_0 = U, R_1 = L R_0 / lb, R_{k+1} = (2/lb) L R_k + R_{k-1}, c_k = (2 -
 * delta_k0) J_k(lb |t_j|) sign(t_j)^k (lb = lambda_bar), truncated at the
 * smallest degree whose dropped coefficients sum to at most cheb_tol.  This
 * is the real form of eq. cheby: on an eigenvector of L with eigenvalue
 * i omega, R_k = i^k T_k(omega/lb) U.  Valid while lambda_bar bounds the
 * spectral radius of L.  Outputs must not alias inputs.  stats as for
 * pa_bdm2_apply_L, plus kmax. */
int pa_bdm2_expL_apply(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *t_host,
                       const double *U_in_dev, double *U_out_dev, void *ws_dev,
                       size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats);
/* out = N(U) for B states (B in [1, 64]): the nonlinearity of Sec. 2.5 on
 * this pair, for every test function w in BDM2 and psi in P1DG
 *   int w . u2 = int u . grad^perp(u^perp . w)
 *                - int_Gamma [[n^perp (u^perp . w)]] . u~ + int (div w) |u|^2 / 2,
 *   int psi eta2 = int grad psi . u eta - int_Gamma [[psi u]] eta~,
 * u^perp = k x u, grad^perp = k x grad, ~ the value of the cell the flow
 * leaves, chosen at every facet quadrature point from the normal flux seen
 * by the edge's first cell (positive: that cell, else the other), eta - b
 * in place of eta when a bottom is set (pa_bdm2_set_bottom).  Quadrature: the collapsed 5 x 5
 * rule in cells (the cell integrands have degree 5), 4-point Gauss-Legendre
 * on every side.  M_u solved as for pa_bdm2_apply_L, M_h exactly.
 * Member-major states in device memory; out must not alias U. */
int pa_bdm2_nonlinear(pa_ctx *ctx, const pa_bdm2 *b, int B, const double *U_dev,
                      double *out_dev, void *ws_dev, size_t ws_bytes,
                      const pa_solve_cfg *cfg, pa_stats *stats);
/* The averaged right-hand side of Sec. 2.2 (eq. vt_discretised) on this
 * pair: Nbar_j = sum_m w_m exp(-s_m L) N(exp(s_m L) U_j) for every member j,
 * the nodes of avg (terms with w_m < weight_cut * max w dropped), every
 * exponential as in pa_bdm2_expL_apply, N as in pa_bdm2_nonlinear.  The
 * (member, node) pairs are processed 64 columns at a time, member-major, in
 * a fixed order (results are reproducible bit for bit).  backward
 * PA_BACKWARD_CLENSHAW (the default): members in groups of up to 64 share
 * one forward basis and one Clenshaw sum (a group narrows so that its
 * 2 (kmax + 1) basis and sum vectors a member stay within 32 GiB); per term:
 * every node's exponentials on its own column.  stats: solves,
 * cg_iters, kmax, terms (columns evaluated), resid_max, device_ms. */
int pa_bdm2_phase_avg_rhs(pa_ctx *ctx, const pa_bdm2 *b, const pa_avg *avg, int members,
                          const double *U_dev, double *Nbar_dev, void *ws_dev,
                          size_t ws_bytes, const pa_solve_cfg *cfg, pa_stats *stats);
/* One step dt of the averaged system (Sec. 2.3) for the members' states U
 * (member-major, in place; members in [1, 64]): the Lawson form of RK4,
 *   k1 = Nbar(U), k2 = Nbar(E (U + h k1)), k3 = Nbar(E U + h k2),
 *   k4 = Nbar(E (E U + dt k3)),
 *   U <- E (E (U + dt/6 k1) + dt/3 (k2 + k3)) + dt/6 k4,
 * E = exp(h L), h = dt/2: the paper's stages with exp(L dt/2) applied
 * before the averages of stages 2 and 4 (it commutes with exp(L s)) and the
 * final exp(L dt) U + dt/6 (exp(L dt) k1 + 2 exp(L h) (k2 + k3) + k4)
 * regrouped by linearity.  Averages as pa_bdm2_phase_avg_rhs, exponentials
 * as pa_bdm2_expL_apply.  Stats summed over the stages (maxima for
 * cg_iters_max, kmax and resid_max). */
int pa_bdm2_step(pa_ctx *ctx, const pa_bdm2 *b, const pa_avg *avg, double dt, int members,
                 double *U_dev, void *ws_dev, size_t ws_bytes, const pa_solve_cfg *cfg,
                 pa_stats *stats);
int pa_bdm2_destroy(pa_bdm2 *b);

#ifdef __cplusplus
}
#endif
#endif
