// Rational (REXI) exponential of libpa (internal): kernel arguments and
// launchers of the batched shifted solves and their combinations.
//
// A complex block holds Bc complex columns per row, row-major
// [row][Bc] of double2 (re, im).  Column col = member * P + pole for the P
// independent poles of a call; columns past P * members are padding and stay
// inactive.  The shifted system of pole X (Sec. 2.4, rational form) is solved
// through its velocity Schur complement
//   S y_u = f,  S = a M_u + b F + c G,  a = X, b = -i/lb, c = -gH/(lb^2 X),
//   G = D' A^-1 D (the grad-div matrix on the ELL pattern of M_u, with the
//   operators),
//   f = M_u U_u + q D' U_eta,  q = -i g/(lb X),
// and y_eta = U_eta / X + h A^-1 D y_u with h = i H/(lb X).
#pragma once
#include <hip/hip_runtime.h>

#include "pa_kernels.h"

namespace pa {

// Per complex column (Bc entries each): the Schur coefficients of its pole.
struct RexiCoef {
  const double2 *a, *c, *q, *h, *xinv;
};

// Right-hand sides: column col takes member col / P of a real member block
// [n][Bm] (forward solves, expL), or its own column of a complex block
// [n][Bc] (backward solves).
struct RexiSrc {
  const double *real_blk = nullptr;
  const double2 *cplx_blk = nullptr;
  int Bm = 0;
};

// Per-column BiCGStab state (Bc entries each).
struct RexiState {
  double2 *rho, *alpha, *omega, *beta;
  double *bb;    // |D^-1 f|^2 (preconditioned start residual)
  double *ff;    // |f|^2
  double *tau2;  // squared relative target of the preconditioned residual
  double *res2;  // |f - S x|^2 of the last check
  int *active, *iters, *fresh, *restarts;
  int *fail;     // 1 word: columns that broke down or ran out of iterations
};

struct RexiArgs {
  DevOps ops;
  int Bc, P, ncols;
  double binv;      // 1 / lambda_bar
  RexiCoef co;
  RexiSrc src;
  // velocity blocks [ne][Bc]; p and v are double-buffered by iteration:
  // an iteration reads p, v and writes p_next, v_next (the engine swaps them)
  double2 *x, *r, *p, *v, *p_next, *v_next, *s, *t;
  double *part;                    // per-workgroup partials [wg][nq][Bc]
  int max_wg;
  RexiState st;
  // left preconditioner: D^-1 (Jacobi, lp == nullptr) or P / X with P the
  // learned approximate inverse of M_u (column-major ELL [slot][row] of
  // packed (column, FP32 value), lpw slots).  With P the gathering kernels
  // write the unpreconditioned vector to w and k_rexi_lp applies P / X.
  const uint2 *lp;
  int lpw;
  double2 *w;
  uint32_t seed;   // shadow residual (a counter hash of row and column)
  int mode;        // init kernel: 0 start from x = 0, 1 check and restart
  double rtol2;    // squared relative tolerance of the true residual
  int maxit;
};

// Depth rows of the solution: y_eta = xinv src_eta + h (D y_u) / |c| into
// Yeta [nc][Bc].
struct RexiEtaArgs {
  DevOps ops;
  int Bc, P, ncols;
  RexiCoef co;
  RexiSrc src;
  const double2 *yu;
  double2 *yeta;
};

// out[row][mem Go + m] = sum_{j<P} Re(C[cm][m][j] Y[row][mem P + j]) over the
// rows of a complex block Y [n][Bc] (cm = mem with per-member tables, else
// 0): the forward shifted states of the average, or expL's results.
struct RexiCombineArgs {
  int n, Bc, P, members, Go, Mo, per_member;
  const double2 *Y;
  const double2 *C;  // [cm][Go][P]
  double *out;       // [n][ostride]: columns past members Go are zeroed
  int ostride;
};

// Z[row][mem P + j] = sum_{m<Mi} Cb[m][j] Yn[row][mem Gi + m]: the complex
// right-hand sides of the backward sum.
struct RexiBackArgs {
  int n, Bc, P, members, Gi, Mi, istride;
  const double *Yn;  // [n][istride], member mem's terms from column mem Gi
  const double2 *C;  // [Mi][P]
  double2 *Z;        // [n][Bc]
};

void launch_rexi_init(const RexiArgs &a, hipStream_t s);
void launch_rexi_fin_init(const RexiArgs &a, int nwg, hipStream_t s);
// p_next = r + beta (p - omega v), then v_next = D^-1 S p_next (two kernels)
void launch_rexi_v(const RexiArgs &a, hipStream_t s);
void launch_rexi_fin_v(const RexiArgs &a, int nwg, hipStream_t s);
void launch_rexi_t(const RexiArgs &a, hipStream_t s);
void launch_rexi_fin_t(const RexiArgs &a, int nwg, hipStream_t s);
void launch_rexi_x(const RexiArgs &a, hipStream_t s);
void launch_rexi_fin_x(const RexiArgs &a, int nwg, hipStream_t s);
// y = P w / X into the kernel's output with its partials (learned form):
// kind 0 after init (r = y, p = y; |w|^2, |y|^2, (r~, y)), 1 after the
// direction product (v_next = y; (r~, y)), 2 after s (t = y; (y, s), |y|^2)
void launch_rexi_lp(const RexiArgs &a, int kind, hipStream_t s);
int rexi_grid(int ne, int Bc);  // workgroups of the row kernels
void launch_rexi_eta(const RexiEtaArgs &a, hipStream_t s);
void launch_rexi_combine(const RexiCombineArgs &a, hipStream_t s);
void launch_rexi_back(const RexiBackArgs &a, hipStream_t s);

}  // namespace pa
