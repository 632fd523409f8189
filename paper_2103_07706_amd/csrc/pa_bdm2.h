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

struct B2Dev {
  int nu = 0, nh = 0, nc = 0;
  double g = 0;
  const int32_t *col = nullptr;    // [kB2W][nu] column-major
  const double *mass = nullptr;    // [kB2W][nu]
  const double *cor = nullptr;     // [kB2W][nu]
  const int32_t *bcol = nullptr;   // [kB2WB][nu]
  const double *bval = nullptr;    // [kB2WB][nu]
  const double *dinv = nullptr;    // [nu]
  const int32_t *cdof = nullptr;   // [nc][12] velocity unknowns of each cell
  const double *q = nullptr;       // [nc][3][12]: -H M_h^-1 B^T of the cell
};

// Per-launch arguments; blocks are row-major [row][Bs].
struct B2Args {
  B2Dev d;
  int Bs;
  double scale;
  const double *u, *eta;          // input state (velocity rows, depth rows)
  const double *addu, *adde;      // addends (nullable): x_0 of the solve, depth
  double *x, *r, *dir;            // solve: iterate, residual, direction
  double *eta_out;
  double c1, c2, theta_inv;
  const double *dir_in;
  double *dir_out;
  int last;
  double *part;                   // per-workgroup partials [wg][Bs]
  double *norms;                  // [2][Bs]: |r_0|^2, |r_K|^2
  double rtol2;
  int *fail;
  unsigned long long *rmax;       // largest relative final residual (bits of a double)
  // accumulation acc += coef[col] * (u, eta)
  double *acc;
  const double *coef;
};

void launch_b2_stiff(const B2Args &a, hipStream_t s);
void launch_b2_step(const B2Args &a, hipStream_t s);
void launch_b2_norm(const B2Args &a, int slot, hipStream_t s);  // partials of |r|^2 -> norms[slot]
void launch_b2_check(const B2Args &a, hipStream_t s);
void launch_b2_acc(const B2Args &a, hipStream_t s);
int b2_grid(int rows, int Bs);

}  // namespace pa

struct pa_bdm2 {
  const pa_mesh *mesh = nullptr;
  int ne = 0, nc = 0, nu = 0, nh = 0;
  double g = 0, H = 0, omega = 0, lambda_bar = 0;
  double eig_min = 0, eig_max = 0;  // Ritz bounds of D^-1 M_u
  std::vector<int32_t> col, bcol, cdof;
  std::vector<double> mass, cor, bval, dinv, q;
  size_t dev_bytes = 0;
  void *dev = nullptr;
  pa::B2Dev d;
};
