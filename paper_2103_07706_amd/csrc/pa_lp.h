// Learned mass-matrix preconditioner (internal): graph tables, network
// kernels (forward, backward, probe loss, Adam) and host helpers.
//
// Network (width 32, relu, three rounds of edge -> cell -> edge messages on
// the edge-cell graph), heads and loss are defined in include/pa.h; the
// kernels below follow that definition.
#pragma once
#include <hip/hip_runtime.h>

#include "pa_internal.h"

struct pa_lp {
  std::vector<float> theta;  // parameters in storage order
};

namespace pa {

constexpr int kLpW = 32;
constexpr int kLpFE = 8, kLpFC = 4, kLpFPad = 8;
constexpr int kLpLayers = 3;
constexpr int kLpProbeMax = 16;

// Offsets (floats) of the parameters in storage order; each weight matrix is
// [inputs][outputs], row-major.
struct LpLayout {
  int ee_W, ee_b, ce_W, ce_b;
  int cl_W[kLpLayers], cl_b[kLpLayers], el_W[kLpLayers], el_b[kLpLayers];
  int hd_w, hd_b, p1_W, p1_b, p2_w, p2_b;
  int total;
};
LpLayout lp_layout();
std::vector<float> lp_init_params(uint64_t seed);

// Host tables of one operator's graph (library numbering).  Pairs are the
// off-diagonal mass-pattern entries p = 4 i + s (slot s + 1 of row i).
struct LpGraphHost {
  int ne = 0, nc = 0;
  std::vector<float> Fe, Fc;             // [ne][8], [nc][8] (4 features + zeros)
  std::vector<int32_t> ce, ec;           // [nc][3], [ne][2]
  std::vector<int32_t> pj, pc, tpos;     // [4 ne]: column, shared cell, transposed pair
  std::vector<int32_t> revc;             // [nc][6]: pairs whose shared cell is c
  std::vector<double> mhat;              // [4 ne]: D^-1/2 M D^-1/2 off the diagonal
  std::vector<int32_t> mcol;             // [ne][5]
  std::vector<double> mval;              // [ne][5], scaled
};
LpGraphHost lp_graph(const pa_ops *o);

struct LpGraphDev {
  int ne = 0, nc = 0;
  const float *Fe = nullptr, *Fc = nullptr;
  const int32_t *ce = nullptr, *ec = nullptr, *pj = nullptr, *pc = nullptr, *tpos = nullptr;
  const int32_t *revc = nullptr, *mcol = nullptr;
  const double *mhat = nullptr, *mval = nullptr;
};

enum { LP_ENC_E = 0, LP_ENC_C = 1, LP_CELL = 2, LP_EDGE = 3, LP_PAIR = 4 };

// Dense layer Y = relu(X W + b) with X gathered per kind:
//   ENC_E: Fe;  ENC_C: Fc;  CELL: [hA, mean of hB over the 3 edges];
//   EDGE: [hA, mean of hB over the 2 cells];  PAIR: [hA_i, hA_j, hB_c].
struct LpDenseArgs {
  LpGraphDev g;
  int N;
  const float *W, *b;
  const float *hA, *hB;
  float *Y;          // forward output [N][32]
  const float *dY;   // backward: gradient of Y (mask Y > 0 applied inside)
  float *dX;         // backward: gradient of X [N][K]
  double *part;      // weight gradient partials [wg][K*32 + 32]
};

struct LpHeadArgs {
  LpGraphDev g;
  const float *he, *z;     // last edge activations, pair hidden layer
  const float *w_hd, *b_hd, *w_p2, *b_p2;
  double *gam, *gd, *goff; // forward outputs
  double *ddiag, *doff;    // backward: dL/dGhat in, dL/dgamma and dL/dbeta out (in place)
  float *dhe, *dz;         // backward outputs: head part of dL/dhe, dL/dz
};

// Weighted column sums for the head weights: part[wg][o] = sum s_n X[n][o],
// part[wg][32] = sum s_n.
struct LpVgradArgs {
  int N;
  const float *X;
  const double *s;
  double *part;
};

struct LpProbeArgs {
  LpGraphDev g;
  int P;
  const double *gd, *goff;
  const double *in, *z, *zinv;  // zinv[p] = 1 / |z_p|^2
  double *out, *res;
  double *part;                  // loss partials
  int transpose;
};

struct LpGhatGradArgs {
  LpGraphDev g;
  int P;
  const double *w, *res, *u, *z, *zinv;
  double *ddiag, *doff;
};

struct LpScatterArgs {
  LpGraphDev g;
  const float *dxp, *dxe, *dxc;
  float *dhe, *dhc;
  int mode;
};
enum { LP_SC_PAIR = 0, LP_SC_CELLS_FROM_EDGES = 1, LP_SC_EDGES = 2, LP_SC_CELLS_DIRECT = 3 };

struct LpAdamArgs {
  int n;
  float *theta;
  const double *grad;
  double *m, *v;
  double lr, b1, b2, eps, c1, c2, gscale;
};

int lp_in_dim(int kind);
int lp_rows(const LpGraphDev &g, int kind);
int lp_wgrad_groups(int N);
void launch_lp_dense_fwd(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s);
void launch_lp_dense_bwd(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s);
void launch_lp_wgrad(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s);
void launch_lp_heads_fwd(const LpHeadArgs &a, hipStream_t s);
void launch_lp_heads_bwd(const LpHeadArgs &a, hipStream_t s);
void launch_lp_vgrad(const LpVgradArgs &a, hipStream_t s);
void launch_lp_wreduce(const double *part, int groups, int width, double *grad, hipStream_t s);
void launch_lp_probe_G(const LpProbeArgs &a, hipStream_t s);
void launch_lp_probe_M(const LpProbeArgs &a, hipStream_t s);
void launch_lp_ghat_grad(const LpGhatGradArgs &a, hipStream_t s);
void launch_lp_scatter(const LpScatterArgs &a, hipStream_t s);
void launch_lp_adam(const LpAdamArgs &a, hipStream_t s);
void launch_lp_rademacher(double *z, int ne, int P, uint64_t seed, hipStream_t s);
void launch_lp_loss_reduce(const double *part, int groups, double *out, hipStream_t s);
int lp_probe_groups(int ne, int P);

// Host side of attaching a trained network to an operator: P = G G^T and
// P M from Ghat (G = D^-1/2 Ghat), their column-major ELL tables, and the
// Ritz bounds of P M.
void lp_build_preconditioner(pa_ops *o, const std::vector<double> &gd,
                             const std::vector<double> &goff);

}  // namespace pa
