// HIP kernels of the BDM2 x P1DG linear operator (the paper's own spaces,
// Sec. 2.5): the stiffness with the mass-solve set-up, Jacobi Chebyshev
// steps on the velocity mass matrix (ELL width 21 in seven blocks of three
// columns, one block-id table per three rows; column-major value tables so
// that consecutive rows read consecutive entries), residual norms and the
// weighted accumulation of the exponential.  Blocks are row-major
// [row][Bs] with Bs a power of two up to 64, one (row, column) per thread in
// a grid-stride loop whose stride is a multiple of Bs, so a thread keeps its
// column; column sums go through per-workgroup partials and a one-workgroup
// finalize (fixed order).
#include <hip/hip_runtime.h>

#include "pa_bdm2.h"

namespace pa {

namespace {
constexpr int kBWG = 256;

// Table reads of a wave-uniform cell, edge or row go through the constant
// address space (scalar loads) when UNI: with 64 columns a wave holds one
// cell, edge or row at all 64 columns (workgroup starts and strides are
// multiples of 64, and the totals are too, so whole waves leave the loops
// together).
template <bool UNI, class T>
struct KPtr {
  using type = const T *;
};
template <class T>
struct KPtr<true, T> {
  using type = const __attribute__((address_space(4))) T *;
};
template <bool UNI, class T>
__device__ inline typename KPtr<UNI, T>::type kp(const T *p) {
  return (typename KPtr<UNI, T>::type)p;
}
template <bool UNI>
__device__ inline int uni(int v) {
  return UNI ? __builtin_amdgcn_readfirstlane(v) : v;
}


// Per-workgroup column sums of v (the thread's column is tid % Bs): a tree
// over the workgroup in a fixed order (strides are multiples of Bs, so each
// addition stays within one column).
__device__ void b2_partial(double v, int Bs, double *part) {
  __shared__ double red[kBWG];
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = kBWG / 2; h >= Bs; h /= 2) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t < Bs) part[(size_t)blockIdx.x * Bs + t] = red[t];
}

__global__ __launch_bounds__(kBWG) void k_b2_stiff(B2Args a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t nvel = (size_t)d.nu * Bs, total = nvel + (size_t)3 * d.nc * Bs;
  const size_t stride = (size_t)gridDim.x * kBWG;
  double rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    if (i < nvel) {
      const int row = (int)(i / Bs), c = (int)(i % Bs);
      double fu = 0.0, be = 0.0;
      if (!a.rhs) {
#pragma unroll
      for (int t = 0; t < kB2WBlk; t++) {
        const size_t col0 = (size_t)3 * d.bid[(size_t)t * (d.nu / 3) + row / 3];
#pragma unroll
        for (int q = 0; q < 3; q++)
          fu = fma(d.cor[(size_t)(3 * t + q) * d.nu + row], a.u[(col0 + q) * Bs + c], fu);
      }
#pragma unroll
      for (int s = 0; s < kB2WB; s++) {
        const size_t k = (size_t)s * d.nu + row;
        be = fma(d.bval[k], a.eta[(size_t)d.bcol[k] * Bs + c], be);
      }
      }
      const double r = a.rhs ? a.rhs[i] : a.scale * (d.g * be - fu);
      a.r[i] = r;
      a.x[i] = a.addu ? a.addu[i] : 0.0;
      a.dir[i] = a.theta_inv * d.dinv[row] * r;
      rr = fma(r, r, rr);
    } else if (!a.rhs) {
      const size_t j = i - nvel;
      const int row = (int)(j / Bs), c = (int)(j % Bs);
      const int cell = row / 3, qq = row % 3;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 12; k++)
        s = fma(d.q[((size_t)cell * 3 + qq) * 12 + k], a.u[(size_t)d.cdof[12 * cell + k] * Bs + c], s);
      a.eta_out[j] = a.scale * s + (a.adde ? a.adde[j] : 0.0);
    }
  }
  b2_partial(rr, Bs, a.part);
}

// Row form, three-term on the increment y (x = x_0 + y, b in r): y_{k+1} =
// y_k + c1 (y_k - y_{k-1}) + c2 D^-1 (b - M y_k) over y_{k-1} (dir_out);
// with a.last the finish: x += y_K and the partials of |b - M y_K|^2.
__global__ __launch_bounds__(kBWG) void k_b2_step3(B2Args a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t nvel = (size_t)d.nu * Bs, stride = (size_t)gridDim.x * kBWG;
  double rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < nvel; i += stride) {
    const int row = (int)(i / Bs), c = (int)(i % Bs);
    double my = 0.0;
#pragma unroll
    for (int t = 0; t < kB2WBlk; t++) {
      const size_t col0 = (size_t)3 * d.bid[(size_t)t * (d.nu / 3) + row / 3];
#pragma unroll
      for (int q = 0; q < 3; q++)
        my = fma(d.mass[(size_t)(3 * t + q) * d.nu + row], a.dir_in[(col0 + q) * Bs + c], my);
    }
    const double yk = a.dir_in[i], res = a.r[i] - my;
    if (!a.last) {
      a.dir_out[i] = yk + a.c1 * (yk - (a.first ? 0.0 : a.dir_out[i])) + a.c2 * d.dinv[row] * res;
    } else {
      a.x[i] += yk;
      rr = fma(res, res, rr);
    }
  }
  if (a.last) b2_partial(rr, Bs, a.part);
}

// Element form of the step, cell pass: loc[12 c + i] = sum_j mT_c[i][j] d[cdof_j].
template <bool UNI>
__global__ __launch_bounds__(kBWG) void k_b2_mel(B2Args a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t total = (size_t)d.nc * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int cell = uni<UNI>((int)(i / Bs)), c = (int)(i % Bs);
    const auto cdof = kp<UNI>(d.cdof + 12 * (size_t)cell);
    double v[12];
#pragma unroll
    for (int j = 0; j < 12; j++) v[j] = a.dir_in[(size_t)cdof[j] * Bs + c];
    const auto M = kp<UNI>(d.mT + (size_t)144 * cell);
#pragma unroll
    for (int r = 0; r < 12; r++) {
      double y = 0.0;
#pragma unroll
      for (int j = 0; j < 12; j++) y = fma(M[12 * r + j], v[j], y);
      a.loc[((size_t)12 * cell + r) * Bs + c] = y;
    }
  }
}

// Element form, three-term row pass on the increment y of the solve (x =
// x_0 + y, b held in r): y_{k+1} = y_k + c1 (y_k - y_{k-1}) + c2 D^-1 (b -
// M y_k), written over y_{k-1} (dir_out); with a.last instead the finish:
// x += y_K and the partials of |b - M y_K|^2.
template <bool UNI>
__global__ __launch_bounds__(kBWG) void k_b2_step3_el(B2Args a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t nvel = (size_t)d.nu * Bs, stride = (size_t)gridDim.x * kBWG;
  double rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < nvel; i += stride) {
    const int row = uni<UNI>((int)(i / Bs)), c = (int)(i % Bs);
    const auto rl = kp<UNI>(d.rloc + 2 * (size_t)row);
    const int p0 = rl[0], p1 = rl[1];
    double my = a.loc[(size_t)p0 * Bs + c];
    if (p1 >= 0) my += a.loc[(size_t)p1 * Bs + c];
    const double yk = a.dir_in[i], res = a.r[i] - my;
    if (!a.last) {
      a.dir_out[i] = yk + a.c1 * (yk - (a.first ? 0.0 : a.dir_out[i])) + a.c2 * kp<UNI>(d.dinv)[row] * res;
    } else {
      a.x[i] += yk;
      rr = fma(res, res, rr);
    }
  }
  if (a.last) b2_partial(rr, Bs, a.part);
}

// Cell form of the three-term step on 64-column blocks: a wave holds one
// cell at all 64 columns and forms its 12 x 12 product against the cell's
// gathered y_k in registers.  It finishes the cell's three interior rows,
// and the three rows of each edge whose first cell (rloc slot 0) it is,
// adding the other cell's three block rows against that cell's gathered
// values.  Each row's sum is the element form's (the first cell's 12-term
// chain, then the second's), so the result is the same bits, without the
// products' round trip through memory (12 values a cell and column written
// and read again) and in one launch instead of two.  Cells are laid over
// the XCDs in eight contiguous ranges (workgroup b runs on XCD b % 8, and
// the grid is a multiple of 8), so the neighbours a cell gathers from are
// mostly in flight on the same XCD and its L2.
__device__ inline double b2fma(double x, double y, double z) { return fma(x, y, z); }
__device__ inline float b2fma(float x, float y, float z) { return fmaf(x, y, z); }

// The cell walk of the cell form: for each row the wave's cell finishes,
// row(g, y_g, (M y)_g) in the table's type T (values of y converted to T).
template <class T, class V, class F>
__device__ __forceinline__ void b2_cells(const B2Dev &d, const T *mtab, const V *y, F &&row) {
  constexpr int Bs = 64, kWaves = kBWG / 64;
  const int xcd = blockIdx.x & 7, per = gridDim.x >> 3;
  const int cpx = (d.nc + 7) >> 3;
  const int c_end = min(d.nc, (xcd + 1) * cpx);
  const size_t total = (size_t)c_end * Bs, stride = (size_t)per * kWaves * Bs;
  const auto rloc = kp<true>(d.rloc);
  const size_t i0 = ((size_t)xcd * cpx + (size_t)(blockIdx.x >> 3) * kWaves) * Bs + threadIdx.x;
  for (size_t i = i0; i < total; i += stride) {
    const int cell = uni<true>((int)(i / Bs)), c = (int)(i % Bs);
    const auto cdof = kp<true>(d.cdof + 12 * (size_t)cell);
    const auto M = kp<true>(mtab + (size_t)144 * cell);
    T v[12];
#pragma unroll
    for (int j = 0; j < 12; j++) v[j] = (T)y[(size_t)cdof[j] * Bs + c];
#pragma unroll
    for (int r = 9; r < 12; r++) {
      T acc = 0;
#pragma unroll
      for (int j = 0; j < 12; j++) acc = b2fma(M[12 * r + j], v[j], acc);
      row(cdof[r], v[r], acc);
    }
    for (int e = 0; e < 3; e++) {
      const int g0 = cdof[3 * e];
      if (rloc[2 * (size_t)g0] != 12 * cell + 3 * e) continue;  // the edge's second cell
      const int o = rloc[2 * (size_t)g0 + 1];
      const int oc = o >= 0 ? o / 12 : cell;
      const auto ocd = kp<true>(d.cdof + 12 * (size_t)oc);
      const auto OM = kp<true>(mtab + (size_t)144 * oc);
      T w[12];
      if (o >= 0) {
#pragma unroll
        for (int j = 0; j < 12; j++) w[j] = (T)y[(size_t)ocd[j] * Bs + c];
      }
#pragma unroll
      for (int q = 0; q < 3; q++) {
        const int g = cdof[3 * e + q];
        T acc = 0;
#pragma unroll
        for (int j = 0; j < 12; j++) acc = b2fma(M[12 * (3 * e + q) + j], v[j], acc);
        if (o >= 0) {
          const int os = rloc[2 * (size_t)g + 1] - 12 * oc;
          T z = 0;
#pragma unroll
          for (int j = 0; j < 12; j++) z = b2fma(OM[12 * os + j], w[j], z);
          acc += z;
        }
        row(g, v[3 * e + q], acc);
      }
    }
  }
}

__global__ __launch_bounds__(kBWG) void k_b2_cstep(B2Args a) {
  const auto dinv = kp<true>(a.d.dinv);
  double rr = 0.0;
  b2_cells(a.d, a.d.mT, a.dir_in, [&](int g, double yk, double my) {
    const size_t gi = (size_t)g * 64 + threadIdx.x % 64;
    const double res = a.r[gi] - my;
    if (!a.last) {
      a.dir_out[gi] = yk + a.c1 * (yk - (a.first ? 0.0 : a.dir_out[gi])) + a.c2 * dinv[g] * res;
    } else {
      a.x[gi] += yk;
      rr = fma(res, res, rr);
    }
  });
  if (a.last) b2_partial(rr, 64, a.part);
}

// FP32 inner solves of a 64-column FP64 solve (iterative refinement).
// Start of the first round, rows in order: b32 = (float) r, y_1 = D^-1 b32
// / theta.
__global__ __launch_bounds__(kBWG) void k_b2_mix_init(B2MixArgs a) {
  const size_t total = (size_t)a.d.nu * 64, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const float b = (float)a.r[i];
    a.r32[i] = b;
    a.y_out[i] = (float)a.d.dinv[i / 64] * b * a.theta_inv;
  }
}

// Inner step in FP32, cell form with the FP32 cell blocks: y_{k+1} = y_k +
// c1 (y_k - y_{k-1}) + c2 D^-1 (b32 - M y_k) over y_{k-1} (y_out).
__global__ __launch_bounds__(kBWG) void k_b2_cstep32(B2MixArgs a) {
  const auto dinv = kp<true>(a.d.dinv);
  b2_cells(a.d, a.d.mT32, a.y_cur, [&](int g, float yk, float my) {
    const size_t gi = (size_t)g * 64 + threadIdx.x % 64;
    const float res = a.r32[gi] - my;
    const float yp = a.zero_prev ? 0.0f : a.y_out[gi];
    a.y_out[gi] = yk + a.c1 * (yk - yp) + a.c2 * (float)dinv[g] * res;
  });
}

// End of a round, FP64 cell form: x += y (the round's increment, y_cur),
// r -= M y with the FP64 blocks; then the next round's b32 = (float) r and
// y_1 = D^-1 b32 / theta (y_out), or on the last round the partials of
// |r|^2 for the check.
__global__ __launch_bounds__(kBWG) void k_b2_refine(B2MixArgs a) {
  const auto dinv = kp<true>(a.d.dinv);
  double rr = 0.0;
  b2_cells(a.d, a.d.mT, a.y_cur, [&](int g, double yk, double my) {
    const size_t gi = (size_t)g * 64 + threadIdx.x % 64;
    a.x[gi] += yk;
    const double rn = a.r[gi] - my;
    a.r[gi] = rn;
    if (a.last) {
      rr = fma(rn, rn, rr);
    } else {
      const float b = (float)rn;
      a.r32[gi] = b;
      a.y_out[gi] = (float)dinv[g] * b * a.theta_inv;
    }
  });
  if (a.last) b2_partial(rr, 64, a.part);
}

__global__ __launch_bounds__(kBWG) void k_b2_norm(B2Args a) {
  const int Bs = a.Bs;
  const size_t nvel = (size_t)a.d.nu * Bs, stride = (size_t)gridDim.x * kBWG;
  double rr = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < nvel; i += stride) rr = fma(a.r[i], a.r[i], rr);
  b2_partial(rr, Bs, a.part);
}

// norms[slot][c] = sum of the partials; slot 1 also checks the solve
// (|r_K|^2 <= rtol^2 |r_0|^2, NaN fails) and keeps the largest relative
// residual (non-negative doubles order as their bit patterns).
// One workgroup of kFinT threads: column c = t % Bs, group t / Bs sums the
// partials w = group, group + G, ... with four interleaved accumulators,
// then the groups are added in a fixed tree (the order never changes).
constexpr int kFinT = 1024;
__global__ __launch_bounds__(kFinT) void k_b2_fin(B2Args a, int nwg, int slot) {
  __shared__ double red[kFinT];
  const int t = threadIdx.x, Bs = a.Bs, G = kFinT / Bs, grp = t / Bs, c = t % Bs;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int w = grp;
  for (; w + 3 * G < nwg; w += 4 * G) {
    s0 += a.part[(size_t)w * Bs + c];
    s1 += a.part[(size_t)(w + G) * Bs + c];
    s2 += a.part[(size_t)(w + 2 * G) * Bs + c];
    s3 += a.part[(size_t)(w + 3 * G) * Bs + c];
  }
  for (; w < nwg; w += G) s0 += a.part[(size_t)w * Bs + c];
  red[t] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = G / 2; h >= 1; h /= 2) {
    if (grp < h) red[t] += red[t + h * Bs];
    __syncthreads();
  }
  if (grp != 0) return;
  const double s = red[c];
  a.norms[slot * Bs + c] = s;
  if (slot == 1) {
    const double r0 = a.norms[c];
    if (!(s <= a.rtol2 * r0)) atomicAdd(a.fail, 1);
    const double rel = r0 > 0.0 ? sqrt(s / r0) : 0.0;
    if (rel == rel) atomicMax(a.rmax, (unsigned long long)__double_as_longlong(rel));
  }
}

// Per-workgroup partials of the energy norm H u' M_u u + g eta' M_h eta
// (M_h per cell: A/12 (I + J)).
__global__ __launch_bounds__(kBWG) void k_b2_wnorm(B2Args a, double H) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t nvel = (size_t)d.nu * Bs, total = nvel + (size_t)d.nh * Bs;
  const size_t stride = (size_t)gridDim.x * kBWG;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int row = (int)(i / Bs), c = (int)(i % Bs);
    if (i < nvel) {
      double mu = 0.0;
#pragma unroll
      for (int t = 0; t < kB2WBlk; t++) {
        const size_t col0 = (size_t)3 * d.bid[(size_t)t * (d.nu / 3) + row / 3];
#pragma unroll
        for (int q = 0; q < 3; q++)
          mu = fma(d.mass[(size_t)(3 * t + q) * d.nu + row], a.u[(col0 + q) * Bs + c], mu);
      }
      acc = fma(H * a.u[i], mu, acc);
    } else {
      const int hr = row - d.nu, cell = hr / 3;
      const double *e = a.eta + (size_t)3 * cell * Bs + c;
      const double sum = e[0] + e[(size_t)Bs] + e[(size_t)2 * Bs];
      const double v = a.eta[(size_t)hr * Bs + c];
      acc = fma(d.g * v, d.ncell[(size_t)kB2NC * cell + kNcA] / 12.0 * (v + sum), acc);
    }
  }
  b2_partial(acc, Bs, a.part);
}

__global__ __launch_bounds__(kBWG) void k_b2_acc(B2Args a) {
  const int Bs = a.Bs;
  const size_t nvel = (size_t)a.d.nu * Bs, total = nvel + (size_t)a.d.nh * Bs;
  const size_t stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int c = (int)(i % Bs);
    const double v = i < nvel ? a.u[i] : a.eta[i - nvel];
    a.acc[i] = fma(a.coef[c], v, a.acc[i]);
  }
}
// ---------------------------------------------------------------- N
// Velocity of a cell (raw coefficients a[12]) at scaled point (xi, et):
// value and, when J is given, its Jacobian J[c][d] = d u_c / d x_d.
__device__ inline void b2_eval(const double *a, double xi, double et, double h, double u[2],
                               double J[2][2]) {
  const double m[6] = {1.0, xi, et, xi * xi, xi * et, et * et};
  u[0] = u[1] = 0.0;
#pragma unroll
  for (int k = 0; k < 6; k++) {
    u[0] = fma(m[k], a[2 * k], u[0]);
    u[1] = fma(m[k], a[2 * k + 1], u[1]);
  }
  if (J) {
    const double mx[6] = {0.0, 1.0, 0.0, 2.0 * xi, et, 0.0};
    const double my[6] = {0.0, 0.0, 1.0, 0.0, xi, 2.0 * et};
#pragma unroll
    for (int c = 0; c < 2; c++) {
      double jx = 0.0, jy = 0.0;
#pragma unroll
      for (int k = 0; k < 6; k++) {
        jx = fma(mx[k], a[2 * k + c], jx);
        jy = fma(my[k], a[2 * k + c], jy);
      }
      J[c][0] = jx / h;
      J[c][1] = jy / h;
    }
  }
}

// Scaled coordinates and barycentric weights of point t of side s of a cell
// (t runs from the edge's first vertex to its second: from local vertex
// s+1 to s+2 in the edge's first cell, the reverse in its second).
template <class TP>
__device__ inline void b2_side_point(TP T, int s, double t, double &xi, double &et, double l[3]) {
  const int v1 = (s + 1) % 3, v2 = (s + 2) % 3;
  const bool first = T[kNcSg + s] > 0.0;
  const int ia = first ? v1 : v2, ib = first ? v2 : v1;
  xi = (1.0 - t) * T[kNcX + 2 * ia] + t * T[kNcX + 2 * ib];
  et = (1.0 - t) * T[kNcX + 2 * ia + 1] + t * T[kNcX + 2 * ib + 1];
  l[0] = l[1] = l[2] = 0.0;
  l[ia] = 1.0 - t;
  l[ib] = t;
}

// raw[12 c + f] = sum_j C[f][j] s_j u[cdof_j]
template <bool UNI>
__global__ __launch_bounds__(kBWG) void k_b2_raw(B2NlArgs a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t total = (size_t)d.nc * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int cell = uni<UNI>((int)(i / Bs)), col = (int)(i % Bs);
    const auto T = kp<UNI>(d.ncell + (size_t)kB2NC * cell);
    const auto cdof = kp<UNI>(d.cdof + 12 * (size_t)cell);
    double v[12];
#pragma unroll
    for (int j = 0; j < 12; j++) {
      const double sg = j < 9 ? T[kNcSg + j / 3] : 1.0;
      v[j] = sg * a.u[(size_t)cdof[j] * Bs + col];
    }
#pragma unroll
    for (int f = 0; f < 12; f++) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 12; j++) s = fma(T[kNcC + 12 * f + j], v[j], s);
      a.raw[((size_t)12 * cell + f) * Bs + col] = s;
    }
  }
}

// Upwind traces at the edges' points: the cell the flow leaves (normal
// flux out of c0 positive: c0, else c1); u as a 3D vector and eta.
template <bool UNI>
__global__ __launch_bounds__(kBWG) void k_b2_edge(B2NlArgs a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t total = (size_t)d.ne * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int e = uni<UNI>((int)(i / Bs)), col = (int)(i % Bs);
    const auto et4 = kp<UNI>(d.etab + 4 * (size_t)e);
    int cc[2], ss[2];
    for (int k = 0; k < 2; k++) {
      cc[k] = et4[2 * k];
      ss[k] = et4[2 * k + 1];
    }
    const auto bot = kp<UNI>(d.bot);
    double ar[2][12], hc[2][3];
    for (int k = 0; k < 2; k++) {
#pragma unroll
      for (int f = 0; f < 12; f++) ar[k][f] = a.raw[((size_t)12 * cc[k] + f) * Bs + col];
#pragma unroll
      for (int r = 0; r < 3; r++)
        hc[k][r] = a.eta[((size_t)3 * cc[k] + r) * Bs + col] - bot[3 * cc[k] + r];
    }
    const auto ftab = kp<UNI>(d.ftab);
    for (int p = 0; p < kB2FQ; p++) {
      const double t = ftab[2 * p];
      double u[2][2], hv[2], e3[2][6], flux0 = 0.0;
      for (int k = 0; k < 2; k++) {
        const auto T = kp<UNI>(d.ncell + (size_t)kB2NC * cc[k]);
        double xi, et, l[3];
        b2_side_point(T, ss[k], t, xi, et, l);
        b2_eval(ar[k], xi, et, T[kNcH], u[k], nullptr);
        hv[k] = l[0] * hc[k][0] + l[1] * hc[k][1] + l[2] * hc[k][2];
        if (k == 0) flux0 = u[0][0] * T[kNcNo + 2 * ss[0]] + u[0][1] * T[kNcNo + 2 * ss[0] + 1];
#pragma unroll
        for (int dd = 0; dd < 3; dd++) {
          e3[k][dd] = T[kNcE1 + dd];
          e3[k][3 + dd] = T[kNcE2 + dd];
        }
      }
      // the upwind side differs from column to column: select, per lane,
      // between the two cells' values
      const int w = flux0 > 0.0 ? 0 : 1;
      double *o = a.ut + ((size_t)(e * kB2FQ + p) * 4) * Bs + col;
#pragma unroll
      for (int dd = 0; dd < 3; dd++) o[(size_t)dd * Bs] = u[w][0] * e3[w][dd] + u[w][1] * e3[w][3 + dd];
      o[(size_t)3 * Bs] = hv[w];
    }
  }
}

// Cell integrals: velocity contributions per cell slot (signed), depth rows
// of N (the block-diagonal M_h solved in closed form).
template <bool UNI>
__global__ __launch_bounds__(kBWG) void k_b2_cell(B2NlArgs a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t total = (size_t)d.nc * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int cell = uni<UNI>((int)(i / Bs)), col = (int)(i % Bs);
    const auto T = kp<UNI>(d.ncell + (size_t)kB2NC * cell);
    const auto qtab = kp<UNI>(d.qtab);
    const auto ftab = kp<UNI>(d.ftab);
    const auto bot = kp<UNI>(d.bot);
    const auto cdof = kp<UNI>(d.cdof + 12 * (size_t)cell);
    const double h = T[kNcH], A = T[kNcA];
    double ar[12], hc[3], g[12], rh[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < 12; f++) {
      ar[f] = a.raw[((size_t)12 * cell + f) * Bs + col];
      g[f] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < 3; r++) hc[r] = a.eta[((size_t)3 * cell + r) * Bs + col] - bot[3 * cell + r];
    // volume: u . grad^perp(u^perp . m_a e_c) + (div m_a e_c) |u|^2 / 2
    for (int q = 0; q < kB2VQ; q++) {
      const double l0 = qtab[4 * q], l1 = qtab[4 * q + 1], l2 = qtab[4 * q + 2];
      const double w = qtab[4 * q + 3] * A;
      const double xi = l0 * T[kNcX] + l1 * T[kNcX + 2] + l2 * T[kNcX + 4];
      const double et = l0 * T[kNcX + 1] + l1 * T[kNcX + 3] + l2 * T[kNcX + 5];
      double u[2], J[2][2];
      b2_eval(ar, xi, et, h, u, J);
      const double up[2] = {-u[1], u[0]};
      const double Jp[2][2] = {{-J[1][0], -J[1][1]}, {J[0][0], J[0][1]}};
      const double ke = 0.5 * (u[0] * u[0] + u[1] * u[1]);
      const double m[6] = {1.0, xi, et, xi * xi, xi * et, et * et};
      const double mx[6] = {0.0, 1.0 / h, 0.0, 2.0 * xi / h, et / h, 0.0};
      const double my[6] = {0.0, 0.0, 1.0 / h, 0.0, xi / h, 2.0 * et / h};
#pragma unroll
      for (int k = 0; k < 6; k++) {
#pragma unroll
        for (int c = 0; c < 2; c++) {
          const double gx = Jp[c][0] * m[k] + up[c] * mx[k];
          const double gy = Jp[c][1] * m[k] + up[c] * my[k];
          const double dv = c == 0 ? mx[k] : my[k];
          g[2 * k + c] = fma(w, -u[0] * gy + u[1] * gx + dv * ke, g[2 * k + c]);
        }
      }
      const double hq = l0 * hc[0] + l1 * hc[1] + l2 * hc[2];
#pragma unroll
      for (int r = 0; r < 3; r++)
        rh[r] = fma(w * hq, T[kNcGl + 2 * r] * u[0] + T[kNcGl + 2 * r + 1] * u[1], rh[r]);
    }
    // sides: - |s| w_p ((k x n_out) . u~)(u^perp . m_a e_c) and
    //        - |s| w_p l_r (u . n_out) eta~
    for (int s = 0; s < 3; s++) {
      const int e = cdof[3 * s] / 3;
      const double len = T[kNcLen + s];
      for (int p = 0; p < kB2FQ; p++) {
        const double t = ftab[2 * p], wl = len * ftab[2 * p + 1];
        double xi, et, l[3], u[2];
        b2_side_point(T, s, t, xi, et, l);
        b2_eval(ar, xi, et, h, u, nullptr);
        const double *o = a.ut + ((size_t)(e * kB2FQ + p) * 4) * Bs + col;
        const double sv = T[kNcNp + 3 * s] * o[0] + T[kNcNp + 3 * s + 1] * o[(size_t)Bs] +
                          T[kNcNp + 3 * s + 2] * o[(size_t)2 * Bs];
        const double ht = o[(size_t)3 * Bs];
        const double flux = u[0] * T[kNcNo + 2 * s] + u[1] * T[kNcNo + 2 * s + 1];
        const double up[2] = {-u[1], u[0]};
        const double m[6] = {1.0, xi, et, xi * xi, xi * et, et * et};
#pragma unroll
        for (int k = 0; k < 6; k++) {
          g[2 * k] = fma(-wl * sv, up[0] * m[k], g[2 * k]);
          g[2 * k + 1] = fma(-wl * sv, up[1] * m[k], g[2 * k + 1]);
        }
#pragma unroll
        for (int r = 0; r < 3; r++) rh[r] = fma(-wl * flux * ht, l[r], rh[r]);
      }
    }
    // velocity: slot j gets s_j sum_f C[f][j] g[f]
#pragma unroll
    for (int j = 0; j < 12; j++) {
      double v = 0.0;
#pragma unroll
      for (int f = 0; f < 12; f++) v = fma(T[kNcC + 12 * f + j], g[f], v);
      const double sg = j < 9 ? T[kNcSg + j / 3] : 1.0;
      a.loc[((size_t)12 * cell + j) * Bs + col] = sg * v;
    }
    // depth: M_h^-1 = (12/A)(I - J/4)
    const double sum = rh[0] + rh[1] + rh[2];
#pragma unroll
    for (int r = 0; r < 3; r++) a.eta_out[((size_t)3 * cell + r) * Bs + col] = (12.0 / A) * (rh[r] - 0.25 * sum);
  }
}

// rhs[row] = the (one or two) cell slots of the row
__global__ __launch_bounds__(kBWG) void k_b2_gather(B2NlArgs a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t total = (size_t)d.nu * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int row = (int)(i / Bs), col = (int)(i % Bs);
    const int p0 = d.rloc[2 * row], p1 = d.rloc[2 * row + 1];
    double v = a.loc[(size_t)p0 * Bs + col];
    if (p1 >= 0) v += a.loc[(size_t)p1 * Bs + col];
    a.rhs[i] = v;
  }
}
__global__ __launch_bounds__(kBWG) void k_b2_bcast(B2ColArgs a) {
  const size_t total = (size_t)a.n * a.Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int row = (int)(i / a.Bs), c = (int)(i % a.Bs);
    const int m = a.cmem[c];
    a.blk[i] = m >= 0 ? a.U[(size_t)m * a.n + row] : 0.0;
  }
}

// out[j][row] += sum over the columns c of member j of cw[c] src[row][c]
// (columns in increasing order).
__global__ __launch_bounds__(kBWG) void k_b2_wsum(B2ColArgs a) {
  const size_t total = (size_t)a.jn * a.n, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int j = a.jlo + (int)(i / a.n), row = (int)(i % a.n);
    double v = 0.0;
    for (int c = 0; c < a.Bs; c++)
      if (a.cmem[c] == j) v = fma(a.cw[c], a.src[(size_t)row * a.Bs + c], v);
    a.out[(size_t)j * a.n + row] += v;
  }
}
__global__ __launch_bounds__(kBWG) void k_b2_comb(B2BasisArgs a) {
  const size_t total = (size_t)a.n * a.Vs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int row = (int)(i / a.Vs), c = (int)(i % a.Vs);
    const int col = a.col0 + c, j = col / a.Mk, m = col % a.Mk;
    double v = 0.0;
    if (j < a.G)
      for (int k = 0; k <= a.K; k++)
        v = fma(a.cf[(size_t)k * a.Mk + m], a.R[((size_t)k * a.n + row) * a.Gs + j], v);
    a.V[i] = v;
  }
}

__global__ __launch_bounds__(kBWG) void k_b2_zsum(B2BasisArgs a) {
  const int Kp = a.K + 1;
  const size_t total = (size_t)a.n * a.jn * Kp, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < total; i += stride) {
    const int k = (int)(i % Kp);
    const size_t rj = i / Kp;
    const int j = a.jlo + (int)(rj % a.jn), row = (int)(rj / a.jn);
    if (j >= a.G) continue;
    const int m0 = max(0, a.col0 - j * a.Mk), m1 = min(a.Mk, a.col0 + a.Vs - j * a.Mk);
    double v = a.Z[((size_t)k * a.n + row) * a.Gs + j];
    for (int m = m0; m < m1; m++)
      v = fma(a.cb[(size_t)k * a.Mk + m], a.Y[(size_t)row * a.Vs + (j * a.Mk + m - a.col0)], v);
    a.Z[((size_t)k * a.n + row) * a.Gs + j] = v;
  }
}
}  // namespace

void launch_b2_comb(const B2BasisArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_comb, dim3(b2_grid(a.n, a.Vs)), dim3(kBWG), 0, s, a);
}
void launch_b2_zsum(const B2BasisArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_zsum, dim3(b2_grid(a.n, a.jn * (a.K + 1))), dim3(kBWG), 0, s, a);
}

void launch_b2_bcast(const B2ColArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_bcast, dim3(b2_grid(a.n, a.Bs)), dim3(kBWG), 0, s, a);
}
void launch_b2_wsum(const B2ColArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_wsum, dim3(b2_grid(a.n, a.jn)), dim3(kBWG), 0, s, a);
}

void launch_b2_nl(const B2NlArgs &a, hipStream_t s) {
  if (a.Bs == 64) {
    hipLaunchKernelGGL(k_b2_raw<true>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_edge<true>, dim3(b2_grid(a.d.ne, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_cell<true>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_b2_raw<false>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_edge<false>, dim3(b2_grid(a.d.ne, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_cell<false>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
  }
  hipLaunchKernelGGL(k_b2_gather, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
}

int b2_grid(int rows, int Bs) {
  const size_t n = (size_t)rows * Bs;
  size_t g = (n + kBWG - 1) / kBWG;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

void launch_b2_stiff(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_stiff, dim3(b2_grid(a.d.nu + 3 * a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(kFinT), 0, s, a, b2_grid(a.d.nu + 3 * a.d.nc, a.Bs), 0);
}
// After a last step (row or element form, both on b2_grid(nu, Bs) workgroups)
// left the partials of |r_K|^2: the check against |r_0|^2.
void launch_b2_step3(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_step3, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
}
// Workgroups of a step: the cell form's grid is a multiple of 8 (at most
// 2048, the partials' room); the check reads that many partials.
static int b2_step_grid(const B2Args &a) {
  const int g = b2_grid(a.d.nu, a.Bs);
  return a.Bs == 64 ? (g + 7) / 8 * 8 : g;
}
void launch_b2_cstep(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_cstep, dim3(b2_step_grid(a)), dim3(kBWG), 0, s, a);
}
static int b2_mix_grid(const B2MixArgs &a) { return (b2_grid(a.d.nu, 64) + 7) / 8 * 8; }
void launch_b2_mix_init(const B2MixArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_mix_init, dim3(b2_grid(a.d.nu, 64)), dim3(kBWG), 0, s, a);
}
void launch_b2_cstep32(const B2MixArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_cstep32, dim3(b2_mix_grid(a)), dim3(kBWG), 0, s, a);
}
void launch_b2_refine(const B2MixArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_refine, dim3(b2_mix_grid(a)), dim3(kBWG), 0, s, a);
}
void launch_b2_step3_el(const B2Args &a, hipStream_t s) {
  if (a.Bs == 64) {
    hipLaunchKernelGGL(k_b2_mel<true>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_step3_el<true>, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_b2_mel<false>, dim3(b2_grid(a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
    hipLaunchKernelGGL(k_b2_step3_el<false>, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
  }
}
void launch_b2_check(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(kFinT), 0, s, a, b2_step_grid(a), 1);
}
void launch_b2_norm(const B2Args &a, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_norm, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(kFinT), 0, s, a, b2_grid(a.d.nu, a.Bs), slot);
}
void launch_b2_wnorm(const B2Args &a, double H, hipStream_t s) {
  const int g = b2_grid(a.d.nu + a.d.nh, a.Bs);
  hipLaunchKernelGGL(k_b2_wnorm, dim3(g), dim3(kBWG), 0, s, a, H);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(kFinT), 0, s, a, g, 0);
}
void launch_b2_acc(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_acc, dim3(b2_grid(a.d.nu + a.d.nh, a.Bs)), dim3(kBWG), 0, s, a);
}

}  // namespace pa
