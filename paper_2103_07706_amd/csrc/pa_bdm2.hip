// HIP kernels of the BDM2 x P1DG linear operator (the paper's own spaces,
// Sec. 2.5): the stiffness with the mass-solve set-up, Jacobi Chebyshev
// steps on the velocity mass matrix (ELL width 21, column-major tables so
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

// Per-workgroup column sums of v (the thread's column is tid % Bs).
__device__ void b2_partial(double v, int Bs, double *part) {
  __shared__ double red[kBWG];
  red[threadIdx.x] = v;
  __syncthreads();
  if ((int)threadIdx.x < Bs) {
    double s = 0.0;
    for (int t = threadIdx.x; t < kBWG; t += Bs) s += red[t];
    part[(size_t)blockIdx.x * Bs + threadIdx.x] = s;
  }
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
#pragma unroll
      for (int s = 0; s < kB2W; s++) {
        const size_t k = (size_t)s * d.nu + row;
        fu = fma(d.cor[k], a.u[(size_t)d.col[k] * Bs + c], fu);
      }
#pragma unroll
      for (int s = 0; s < kB2WB; s++) {
        const size_t k = (size_t)s * d.nu + row;
        be = fma(d.bval[k], a.eta[(size_t)d.bcol[k] * Bs + c], be);
      }
      const double r = a.scale * (d.g * be - fu);
      a.r[i] = r;
      a.x[i] = a.addu ? a.addu[i] : 0.0;
      a.dir[i] = a.theta_inv * d.dinv[row] * r;
      rr = fma(r, r, rr);
    } else {
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

// x += d, r -= M d, d' = c1 d + c2 D^-1 r (not on the last step).
__global__ __launch_bounds__(kBWG) void k_b2_step(B2Args a) {
  const B2Dev &d = a.d;
  const int Bs = a.Bs;
  const size_t nvel = (size_t)d.nu * Bs, stride = (size_t)gridDim.x * kBWG;
  for (size_t i = (size_t)blockIdx.x * kBWG + threadIdx.x; i < nvel; i += stride) {
    const int row = (int)(i / Bs), c = (int)(i % Bs);
    double md = 0.0;
#pragma unroll
    for (int s = 0; s < kB2W; s++) {
      const size_t k = (size_t)s * d.nu + row;
      md = fma(d.mass[k], a.dir_in[(size_t)d.col[k] * Bs + c], md);
    }
    const double di = a.dir_in[i];
    a.x[i] += di;
    const double r = a.r[i] - md;
    a.r[i] = r;
    if (!a.last) a.dir_out[i] = a.c1 * di + a.c2 * d.dinv[row] * r;
  }
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
__global__ void k_b2_fin(B2Args a, int nwg, int slot) {
  const int c = threadIdx.x;
  if (c >= a.Bs) return;
  double s = 0.0;
  for (int w = 0; w < nwg; w++) s += a.part[(size_t)w * a.Bs + c];
  a.norms[slot * a.Bs + c] = s;
  if (slot == 1) {
    const double r0 = a.norms[c];
    if (!(s <= a.rtol2 * r0)) atomicAdd(a.fail, 1);
    const double rel = r0 > 0.0 ? sqrt(s / r0) : 0.0;
    if (rel == rel) atomicMax(a.rmax, (unsigned long long)__double_as_longlong(rel));
  }
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
}  // namespace

int b2_grid(int rows, int Bs) {
  const size_t n = (size_t)rows * Bs;
  size_t g = (n + kBWG - 1) / kBWG;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

void launch_b2_stiff(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_stiff, dim3(b2_grid(a.d.nu + 3 * a.d.nc, a.Bs)), dim3(kBWG), 0, s, a);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(64), 0, s, a, b2_grid(a.d.nu + 3 * a.d.nc, a.Bs), 0);
}
void launch_b2_step(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_step, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
}
void launch_b2_check(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_norm, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(64), 0, s, a, b2_grid(a.d.nu, a.Bs), 1);
}
void launch_b2_norm(const B2Args &a, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_norm, dim3(b2_grid(a.d.nu, a.Bs)), dim3(kBWG), 0, s, a);
  hipLaunchKernelGGL(k_b2_fin, dim3(1), dim3(64), 0, s, a, b2_grid(a.d.nu, a.Bs), slot);
}
void launch_b2_acc(const B2Args &a, hipStream_t s) {
  hipLaunchKernelGGL(k_b2_acc, dim3(b2_grid(a.d.nu + a.d.nh, a.Bs)), dim3(kBWG), 0, s, a);
}

}  // namespace pa
