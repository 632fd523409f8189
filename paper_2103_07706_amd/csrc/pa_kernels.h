// Kernel argument blocks and launchers of libpa (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "pa_internal.h"

namespace pa {

// Per-workgroup partial column sums: [tiles][max_wg][nq][64].  partA holds
// p.q of the SpMV kernel, partB the (r.z, r.r) pairs of the set-up and update
// kernels (and the energy products).
struct RedBuf {
  double *partA = nullptr, *partB = nullptr;
  int max_wg = 0;
};

// Per-column state of one batched CG solve (arrays of Bs entries).
struct SolveState {
  double *bb, *rz, *alpha, *beta, *resid;
  int *active, *iters;
  // fused small-batch CG: per-column scalars double-buffered by iteration
  // parity so that workgroup 0 can publish them while others still read
  double *rz2, *al2;      // [2][4]: gamma and alpha
  int *act2, *it2;        // [2][4]
  int *cnt;               // [2]: active columns after the last finalize, by parity
  int *budget_fail;       // 1: columns still active when an iteration budget ran out
  int *cheb_fail;         // 1: Chebyshev solves that missed the residual tolerance
  unsigned long long *resid_max;  // 1: largest final relative residual (FP64 bits)
  int *fail;              // 1 (accumulates over solves)
  int *iter_max;          // 1 (accumulates over solves)
  unsigned *prof;         // [3]: active columns summed over launches, work launches,
                          //      columns of last Chebyshev steps
  unsigned *prof_last;    // = prof + 2
  unsigned long long *prof_bytes;  // 1: algorithmic bytes of the profiled launches
};

// Residual check after a Chebyshev solve (a kernel of its own, or folded
// into the next solve's set-up kernel: blocks = tiles x columns/4).
struct CheckArgs {
  int Bs, nwg_init, nwg_last, max_wg;
  const double *part_init, *part_last;
  const int *colK;
  int kneed;
  double rtol2;
  int *fail;
  double *resid;
  unsigned long long *resid_max;
};

struct StiffArgs {
  DevOps ops;
  int Bs;
  const double *in_u, *in_eta;
  double *out_u, *out_eta;
  const double *addA_u, *addA_eta, *addB_u, *addB_eta;
  double scale;
  const int *colK;
  int kneed;
  double *r;
  // Chebyshev solver: also d_0 = theta_inv D^-1 r_0 and partials of r_0.r_0
  double *d0;
  double theta_inv;
  double *part_rr;
  int max_wg;
  // optional grouped accumulation acc += coef * in
  double *acc_u, *acc_eta;
  const double *coef;
  int acc_k, G;
  SolveState st;
  RedBuf rb;
  CheckArgs chk;   // the previous solve's residual check, done by the first
  int chk_blocks;  // chk_blocks workgroups (0: none)
};

struct CgArgs {
  DevOps ops;
  int Bs;
  double *x, *p;
  const double *r_in, *w_in, *s_in;
  double *r_out, *w_out, *s_out;
  const double *part_in;  // partials of the previous kernel (fused mode)
  double *part_out;
  double rtol2;
  int maxit;
  int k;          // iteration index
  int fused;      // Bs <= 4: every workgroup reduces part_in itself
  int nwg_prev, check_only, last_check;
  int count_cols; // measurement hook: tally active columns of each launch
  const int *colK;
  int kneed;
  SolveState st;
  RedBuf rb;
};

// Chebyshev semi-iteration step on the mass matrix (see k_cheb_iter).
struct ChebArgs {
  DevOps ops;
  int Bs;
  double *x, *r;
  const double *d_in;
  double *d_out;
  double c1, c2;
  const int *colK;
  int kneed, last;
  double *part;  // last step: partials of r.r
  int max_wg;
  unsigned *prof;  // measurement hook: [0] active columns, [1] launches, [2] columns of last steps
  int nodir;       // 1: update x and r only (the direction comes from another kernel)
};

// Jacobi Chebyshev solve of a block in three-term form on the increment y
// of x (see k_cheb3_iter): a step forms
//   y_{i+1} = y_i + c1 (y_i - y_{i-1}) + c2 D^-1 (b - M y_i)
// (y_{i-1} = 0 when zero_prev; y_next may alias y_prev); the finishing
// launch (finish = 1) adds x += y_cur and leaves partials of r.r with
// r = b - M y_cur, the true residual of the solve.
struct Cheb3Args {
  DevOps ops;
  int Bs;
  const double *y_cur, *y_prev, *b;
  double *y_next, *x;
  double c1, c2;
  const int *colK;
  int kneed, zero_prev, finish;
  double *part;
  int max_wg;
  unsigned *prof;                  // measurement hook: [0] active columns of steps,
                                   // [1] launches, [2] active columns of finishes
  unsigned long long *prof_bytes;  // algorithmic bytes of the launches added here
};

// S Jacobi Chebyshev steps of a single-column solve in one launch (see
// k_cheb_fused), step s with (c1[s], c2[s]); r and d each move from an input
// to an output buffer (other workgroups still read the inputs).
struct ChebFusedArgs {
  DevOps ops;
  int S;            // 1 <= S <= ops.fused_max
  int slots[kFusedMax];  // per step s: ring slots of kPartRows rows that rings
                        // 1..S-1-s of the largest part fill
  double *x;
  const double *r_in, *d_in;
  double *r_out, *d_out;
  double c1[kFusedMax], c2[kFusedMax];
  const int *colK;
  int kneed, last;  // last: step S is the solve's last (partials of r.r, no direction)
  double *part;
  unsigned *prof;   // measurement hook, as ChebArgs
  unsigned long long *prof_bytes;  // algorithmic bytes of the launch added here
  unsigned long long bytes;
  // setup = 1 (the solve's first launch): step 1 is the set-up of the solve,
  // as k_stiff does it: r_0 = scale (-F u + g D' eta), d_0 = theta_inv D^-1
  // r_0, x_0 = addA_u + addB_u (each addend optional), with partials of
  // r_0.r_0 per workgroup and the depth rows out_eta = scale (-H D u / |c|) +
  // addA_eta + addB_eta on cpp cells per part; steps 2..S are Chebyshev
  // steps with c1[1..S-1], c2[1..S-1]; the previous solve's residual check
  // runs in chk_blocks workgroups added past the last part.  r_in, d_in
  // are not read.
  int setup;
  const double *in_u, *in_eta, *addA_u, *addA_eta, *addB_u, *addB_eta;
  double *out_eta;
  double scale, theta_inv;
  int cpp;
  double *part_rr;
  CheckArgs chk;
  int chk_blocks;
};

// Chebyshev step with the learned preconditioner P (see k_cheb_lp_iter):
// residuals ping-pong between r_in and r_out.
struct ChebLpArgs {
  DevOps ops;
  DevLp lp;
  int Bs;
  double *x;
  const double *r_in, *d_in;
  double *r_out, *d_out;
  double c1, c2;
  const int *colK;
  int kneed, last;
  double *part;
  int max_wg;
  unsigned *prof;
};

// d_out = c1 d_in + c2 P r (learned direction; c1 = 0: d_in not read).
struct LpDirArgs {
  DevOps ops;
  DevLp lp;
  int Bs;
  const double *r, *d_in;
  double *d_out;
  double c1, c2;
  const int *colK;
  int kneed;
};

// FP32 inner Chebyshev step (mixed precision), three-term form:
// x_{i+1} = x_i + c1 (x_i - x_{i-1}) + c2 D^-1 (b - M32 x_i), all in FP32.
struct Cheb32Args {
  DevOps ops;
  int Bs;
  const float *x_cur, *x_prev;  // x_i (gathered), x_{i-1} (own row only)
  float *x_next;                // x_{i+1}; may alias x_prev
  const float *b32;             // right-hand side
  float c1, c2;
  const int *colK;
  int kneed, zero_prev;         // zero_prev: x_{i-1} = 0 (not read)
  unsigned *prof;               // measurement hook: [0] active columns, [1] launches
  unsigned long long *prof_bytes;
};

// FP64 refinement: x += x32, r -= M x32 (FP64 matrix), then FP32 copies for
// the next inner solve: its right-hand side r32 = r and its first iterate
// d32 = D^-1 r32 / theta.  first = 1: only the conversion (x32 not yet
// formed, not read).  last = 1: partials of r.r, no copies and r not stored.
struct RefineArgs {
  DevOps ops;
  int Bs;
  double *x, *r;
  const float *x32;
  float *r32, *d32;
  float theta_inv;
  const int *colK;
  int kneed, first, last;
  int x_zero;  // x is still 0 (not read; x = x32 is written)
  double *part;
  int max_wg;
};


enum { FIN_INIT = 0, FIN_STEP = 1, FIN_OUT = 2 };
struct FinArgs {
  int mode, Bs, nwg, max_wg, nq;
  const double *part;
  SolveState st;
  const int *colK;
  int kneed;
  double rtol2;
  int maxit;
  int slot_in, slot_out, slot_zero;
  int last_check;
  double *out;
};

struct CombineArgs {
  int nrows, BsE, BsR, G, members, kmax;
  size_t basis_stride;
  const double *basis, *cf;
  double *E;
};

struct ReduceTermsArgs {
  int nrows, BsY, BsZ, G, kmax;
  size_t zstride;
  const double *Y, *cb;
  double *Z;
};

struct NlArgs {
  DevOps ops;
  int Bs;
  const double *u, *eta;
  double *C, *out_eta;
};

struct GatherArgs {
  DevOps ops;
  int Bs;
  const double *C;
  double *r, *x;
  double *d0;
  double theta_inv;
  // FP32-refined solve next: its first inner right-hand side r32 = r and
  // first iterate x1_32 = D^-1 r32 / theta (what the first refinement
  // kernel would write); d0 is then not written
  float *r32, *x1_32;
  float theta_inv32;
  double *part_rr;  // partials of r.r (solves with a residual check)
  int max_wg;
  const int *colK;
  int kneed;
  SolveState st;
  RedBuf rb;
  CheckArgs chk;   // as in StiffArgs
  int chk_blocks;
};

struct AccArgs {
  int nrows, Bs, G, acc_k;
  const double *in, *coef;
  const int *colK;
  double *acc;
};

struct AxpyArgs {
  size_t n;
  double a0, a1, a2;
  const double *x0, *x1, *x2;
  double *out;
};

struct TransArgs {
  int n, B, Bs;
  double *states, *blk;
};

struct DiagArgs {
  DevOps ops;
  int Bs;
  double H;
  const double *u, *eta;
  double *part;
  int max_wg;
};

int launch_max_wg();
// Measurement hook: the next launch of a profiled kernel (Chebyshev, learned
// and CG steps) records e0 and e1 as part of its dispatch, so that their
// elapsed time is the kernel's own duration.
void arm_launch_events(hipEvent_t e0, hipEvent_t e1);
bool launch_events_armed();
// the launch shape in force for the calling thread (the enclosing
// TuneScope's, else the process default)
LaunchTune launch_tuning();
int launch_rows_grid(int rows, int Bs);
void launch_finalize(const FinArgs &a, hipStream_t s);
void launch_stiff(const StiffArgs &a, hipStream_t s);
void launch_cg_init(const CgArgs &a, hipStream_t s);
void launch_cheb_iter(const ChebArgs &a, hipStream_t s);
void launch_cheb3_iter(const Cheb3Args &a, hipStream_t s);
void launch_cheb_fused(const ChebFusedArgs &a, hipStream_t s);
// workgroups of k_cheb_fused with `extra` workgroups past the last part (0: not available)
int cheb_fused_grid(const DevOps &o, int extra = 0);
void launch_cheb_check(const CheckArgs &a, hipStream_t s);
int cheb_check_blocks(const CheckArgs &a);  // workgroups of a residual check
void launch_cheb_lp_iter(const ChebLpArgs &a, hipStream_t s);
void launch_lp_dir(const LpDirArgs &a, hipStream_t s);
void launch_cheb32_iter(const Cheb32Args &a, hipStream_t s);
void launch_refine(const RefineArgs &a, hipStream_t s);
void launch_cg_iter(const CgArgs &a, hipStream_t s);
void launch_combine(const CombineArgs &a, hipStream_t s);
void launch_reduce_terms(const ReduceTermsArgs &a, hipStream_t s);
void launch_nl_cell(const NlArgs &a, hipStream_t s);
void launch_nl_gather(const GatherArgs &a, hipStream_t s);
void launch_acc(const AccArgs &a, hipStream_t s);
void launch_axpy(const AxpyArgs &a, hipStream_t s);
void launch_to_block(const TransArgs &a, hipStream_t s);
void launch_from_block(const TransArgs &a, hipStream_t s);
void launch_diag(const DiagArgs &a, hipStream_t s);
void launch_zero(unsigned *p, size_t n, hipStream_t s);

}  // namespace pa
