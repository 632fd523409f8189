// The paper's own pair of spaces (Sec. 2.5): BDM2 velocity x P1DG depth,
// linear operator and Chebyshev exponential (internal declarations).
//
// Velocity unknowns: the normal component at the three Gauss points of
// every edge (3 e + k, points ordered from the edge's first vertex to its
// second, value measured across the edge from its first cell to its
// second), then three interior moments per cell (3 ne + 3 c + m); depth
// unknowns: the three barycentric coefficients of every cell (3 c + q).
#pragma once
#include <hip/hip_runtime.h>

#include "pa_internal.h"

namespace pa {

constexpr int kB2W = 21;   // ELL width of the velocity rows (21 unknowns share a cell with an edge unknown)
constexpr int kB2WB = 6;   // ELL width of the divergence rows (depth unknowns of the adjacent cells)
constexpr int kB2WBlk = 7; // column blocks of three per velocity row (kB2W = 3 kB2WBlk)

// Per-cell table of the nonlinear term, kB2NC doubles a cell: the raw
// coefficients of the dual basis (C[f][j] at 12 f + j: basis function j is
// sum_f C[f][j] m_{f/2} e_{f%2}, m = 1, xi, eta, xi^2, xi eta, eta^2 in the
// scaled coordinates (x - x_T)/h of the cell's frame), the vertices in
// those coordinates, h, the area, the barycentric gradients, e1 and e2
// (3D), per side k x n_out (3D), n_out (frame), the length and the sign of
// the edge (+1: the cell is the edge's first).
constexpr int kB2NC = 192;
enum {
  kNcC = 0, kNcX = 144, kNcH = 150, kNcA = 151, kNcGl = 152, kNcE1 = 158, kNcE2 = 161,
  kNcNp = 164, kNcNo = 173, kNcLen = 179, kNcSg = 182
};
constexpr int kB2VQ = 25;  // volume points (collapsed 5 x 5 rule)
constexpr int kB2FQ = 4;   // points per side (Gauss-Legendre)

struct B2Dev {
  int nu = 0, nh = 0, nc = 0, ne = 0;
  double g = 0;
  const int32_t *bid = nullptr;    // [kB2WBlk][nu / 3]: column blocks of each row block;
                                   // slot s of row r is column 3 bid[s / 3][r / 3] + s % 3
  const double *mass = nullptr;    // [kB2W][nu]
  const double *cor = nullptr;     // [kB2W][nu]
  const int32_t *bcol = nullptr;   // [kB2WB][nu]
  const double *bval = nullptr;    // [kB2WB][nu]
  const double *dinv = nullptr;    // [nu]
  const int32_t *cdof = nullptr;   // [nc][12] velocity unknowns of each cell
  const double *q = nullptr;       // [nc][3][12]: -H M_h^-1 B^T of the cell
  const double *ncell = nullptr;   // [nc][kB2NC]
  const int32_t *etab = nullptr;   // [ne][4]: c0, side in c0, c1, side in c1
  const int32_t *rloc = nullptr;   // [nu][2]: 12 c + slot of the row's cells (-1: none)
  const double *qtab = nullptr;    // [kB2VQ][4]: barycentric l0, l1, l2, weight (sum 1)
  const double *ftab = nullptr;    // [kB2FQ][2]: t in [0, 1], weight (sum 1)
  const double *mT = nullptr;      // [nc][12][12]: s_i s_j (M_u)_T of the cell slots
  const float *mT32 = nullptr;     // [nc][12][12]: the same rounded to FP32 (inner solves)
  const double *bot = nullptr;     // [nh]: bottom height (P1DG coefficients)
};
// Blocks at least this wide take the element form of the mass-solve step
// (a cell pass and a row pass) instead of the row kernel; blocks of 64
// columns take the cell form (one launch, no cell products in memory).
constexpr int kB2ElMin = 8;
// Workspace the shared-basis average may spend on a group's bases and sums
// (the group narrows below 64 members beyond it).
constexpr double kB2BasisBytes = 32.0 * (1ull << 30);

// Per-launch arguments; blocks are row-major [row][Bs].
struct B2Args {
  B2Dev d;
  int Bs;
  double scale;
  const double *u, *eta;          // input state (velocity rows, depth rows)
  const double *addu, *adde;      // addends (nullable): x_0 of the solve, depth
  const double *rhs;              // given velocity right-hand side (nullable;
                                  // then the depth rows are not written)
  double *x, *r, *dir;            // solve: iterate, residual, direction
  double *eta_out;
  double c1, c2, theta_inv;
  const double *dir_in;
  double *dir_out;
  int last;
  int first;                      // three-term step 1: y_0 = 0 (dir_out not read)
  double *part;                   // per-workgroup partials [wg][Bs]
  double *loc;                    // element step: [nc * 12][Bs] cell products
  double *norms;                  // [2][Bs]: |r_0|^2, |r_K|^2
  double rtol2;
  int *fail;
  unsigned long long *rmax;       // largest relative final residual (bits of a double)
  // accumulation acc += coef[col] * (u, eta)
  double *acc;
  const double *coef;
};

// The nonlinear term (one thread per cell or edge and column): raw
// coefficients of the velocity, upwind traces at the edges' points, the
// cell integrals (depth rows written, velocity contributions per cell
// slot), and their sum per velocity row.
struct B2NlArgs {
  B2Dev d;
  int Bs;
  const double *u, *eta;   // input state (velocity rows, depth rows)
  double *raw;             // [nc * 12][Bs]
  double *ut;              // [ne * kB2FQ * 4][Bs]: upwind u (3D), upwind eta
  double *loc;             // [nc * 12][Bs]
  double *rhs;             // [nu][Bs]
  double *eta_out;         // depth rows of N
};
void launch_b2_nl(const B2NlArgs &a, hipStream_t s);

// Columns of an averaging pass: column c holds member cmem[c] (-1:
// padding) at a node of weight cw[c]; members jlo .. jlo + jn - 1 occur.
struct B2ColArgs {
  int n, Bs, jlo, jn;
  const int32_t *cmem;
  const double *cw;
  const double *U;    // member-major states [members][n]
  double *out;        // member-major results, accumulated
  double *blk;        // bcast: [n][Bs] block of the columns' members
  const double *src;  // wsum: [n][Bs] block summed into out with the weights
};
// The average with shared bases (members j < G of a group, kept nodes
// m < Mk, node column j Mk + m; a pass holds the Vs node columns from col0
// on, [n][Vs], and touches members jlo .. jlo + jn - 1; bases and sums
// [k][n][Gs]):
//   comb: V(j, m) = sum_k cf[k][m] R_k[j]        (forward exponentials)
//   zsum: Z_k[j] += sum_m cb[k][m] Y(j, m)       (backward weights, the
//         pass's columns; passes in a fixed order)
struct B2BasisArgs {
  int n, Gs, G, Mk, Vs, col0, jlo, jn, K;
  const double *cf, *cb;   // [K + 1][Mk]
  const double *R;         // comb: bases
  double *V;               // comb: node columns
  const double *Y;         // zsum: N of the node columns
  double *Z;               // zsum: the backward sums
};
void launch_b2_comb(const B2BasisArgs &a, hipStream_t s);
void launch_b2_zsum(const B2BasisArgs &a, hipStream_t s);
void launch_b2_bcast(const B2ColArgs &a, hipStream_t s);
void launch_b2_wsum(const B2ColArgs &a, hipStream_t s);

void launch_b2_stiff(const B2Args &a, hipStream_t s);
// One step of a mass solve in three-term form on the increment y (dir_in =
// y_k, dir_out = y_{k-1} -> y_{k+1}; with last: the finish x += y_K and the
// residual partials), row form (ELL rows), element form (cell pass and
// row pass, for blocks of kB2ElMin to 32 columns) or cell form (64 columns).
void launch_b2_step3(const B2Args &a, hipStream_t s);
void launch_b2_step3_el(const B2Args &a, hipStream_t s);
void launch_b2_cstep(const B2Args &a, hipStream_t s);
// FP32 inner solves with FP64 refinement on 64-column blocks (cell form):
// k_b2_mix_init starts the first round from r; each round runs FP32 steps
// (k_b2_cstep32) and ends in k_b2_refine (x += y, r -= M y in FP64, the
// next round's start or, on the last, the residual partials).
struct B2MixArgs {
  B2Dev d;
  double *x, *r;          // FP64 iterate and residual, [nu][64]
  float *r32;             // FP32 right-hand side of the inner solve
  const float *y_cur;     // step: y_k; refine: the round's increment
  float *y_out;           // step: y_{k-1} -> y_{k+1}; init, refine: the next y_1
  float c1, c2, theta_inv;
  int zero_prev, last;
  double *part;           // refine on the last round: partials of |r|^2
};
void launch_b2_mix_init(const B2MixArgs &a, hipStream_t s);
void launch_b2_cstep32(const B2MixArgs &a, hipStream_t s);
void launch_b2_refine(const B2MixArgs &a, hipStream_t s);
void launch_b2_norm(const B2Args &a, int slot, hipStream_t s);  // partials of |r|^2 -> norms[slot]
void launch_b2_check(const B2Args &a, hipStream_t s);  // after the last step: |r_K|^2 vs rtol^2 |r_0|^2
void launch_b2_acc(const B2Args &a, hipStream_t s);
// norms[0][c] = H u' M_u u + g eta' M_h eta of column c of (u, eta)
void launch_b2_wnorm(const B2Args &a, double H, hipStream_t s);
int b2_grid(int rows, int Bs);

}  // namespace pa

struct pa_bdm2 {
  const pa_mesh *mesh = nullptr;
  int ne = 0, nc = 0, nu = 0, nh = 0;
  double g = 0, H = 0, omega = 0, lambda_bar = 0;
  double eig_min = 0, eig_max = 0;  // Ritz bounds of D^-1 M_u
  std::vector<int32_t> col, bid, bcol, cdof;
  std::vector<double> mass, cor, bval, dinv, q, ncell, qtab, ftab, mT, bot;
  std::vector<float> mT32;
  std::vector<int32_t> etab, rloc;
  size_t dev_bytes = 0;
  void *dev = nullptr;
  pa::B2Dev d;
};
