// Kernels of the learned mass-matrix preconditioner: the message-passing
// network on the edge-cell graph (forward and backward), its probe loss
// ||Ghat^T Mhat Ghat z - z||^2 / ||z||^2 and the Adam update.
//
// Dense layers run on the matrix cores: a wave computes a 32-row x 32-output
// tile with v_mfma_f32_32x32x8bf16_1k (BF16 inputs and weights, FP32
// accumulation) or v_mfma_f32_32x32x2f32 (FP32).  Operand lane layout of
// both: lane l supplies row (l % 32) of A and column (l % 32) of B at inner
// indices 4 (l / 32) + t (BF16, t < 4) or l / 32 (FP32); accumulator register
// q of lane l holds row 8 (q / 4) + 4 (l / 32) + q % 4, column l % 32.
// The layer inputs are gathered on the fly from the activations (concatenation
// and neighbour means), never stored.
#include "pa_lp.h"

namespace pa {
namespace {

constexpr int kLpWG = 256;
typedef short lp_s4 __attribute__((ext_vector_type(4)));
typedef float lp_f16 __attribute__((ext_vector_type(16)));

// round to nearest even
__device__ inline short lp_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <int KIND>
struct LpDims {
  static constexpr int K = KIND == LP_PAIR ? 96 : (KIND == LP_CELL || KIND == LP_EDGE) ? 64 : 8;
  static constexpr int KR = KIND == LP_ENC_C ? kLpFC : K;  // stored weight rows
};

// Element k of the input row n of a dense layer.
template <int KIND>
__device__ inline float lp_x(const LpDenseArgs &a, int n, int k) {
  if (KIND == LP_ENC_E) return a.g.Fe[(size_t)n * kLpFPad + k];
  if (KIND == LP_ENC_C) return a.g.Fc[(size_t)n * kLpFPad + k];
  if (KIND == LP_CELL) {
    if (k < 32) return a.hA[(size_t)n * 32 + k];
    const int32_t *e = a.g.ce + 3 * (size_t)n;
    k -= 32;
    return (a.hB[(size_t)e[0] * 32 + k] + a.hB[(size_t)e[1] * 32 + k] + a.hB[(size_t)e[2] * 32 + k]) *
           (1.0f / 3.0f);
  }
  if (KIND == LP_EDGE) {
    if (k < 32) return a.hA[(size_t)n * 32 + k];
    const int32_t *c = a.g.ec + 2 * (size_t)n;
    k -= 32;
    return 0.5f * (a.hB[(size_t)c[0] * 32 + k] + a.hB[(size_t)c[1] * 32 + k]);
  }
  if (k < 32) return a.hA[(size_t)(n >> 2) * 32 + k];
  if (k < 64) return a.hA[(size_t)a.g.pj[n] * 32 + k - 32];
  return a.hB[(size_t)a.g.pc[n] * 32 + k - 64];
}

__device__ inline void lp_zero(lp_f16 &v) {
#pragma unroll
  for (int q = 0; q < 16; q++) v[q] = 0.0f;
}

// accumulator register q -> row offset inside the 32 x 32 tile
__device__ inline int lp_acc_row(int q, int half) { return (q >> 2) * 8 + half * 4 + (q & 3); }

// Y = relu(X W + b); one wave per 32 rows, four waves per workgroup.
template <int KIND, bool BF16>
__global__ __launch_bounds__(kLpWG) void k_lp_dense_fwd(LpDenseArgs a) {
  constexpr int K = LpDims<KIND>::K, KR = LpDims<KIND>::KR;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int row0 = (blockIdx.x * 4 + wave) * 32;
  if (row0 >= a.N) return;  // whole wave
  const int r = row0 + col;
  const bool rv = r < a.N;
  lp_f16 acc;
  lp_zero(acc);
  if constexpr (BF16) {
    for (int k0 = 0; k0 < K; k0 += 8) {
      lp_s4 av, bv;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int k = k0 + 4 * half + t;
        av[t] = lp_bf16(rv && k < KR ? lp_x<KIND>(a, r, k) : 0.0f);
        bv[t] = lp_bf16(k < KR ? a.W[k * 32 + col] : 0.0f);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 2) {
      const int k = k0 + half;
      const float av = rv && k < KR ? lp_x<KIND>(a, r, k) : 0.0f;
      const float bv = k < KR ? a.W[k * 32 + col] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
  }
  const float bias = a.b[col];
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int row = row0 + lp_acc_row(q, half);
    if (row < a.N) a.Y[(size_t)row * 32 + col] = fmaxf(acc[q] + bias, 0.0f);
  }
}

// dPre = dY (.) [Y > 0]
__device__ inline float lp_dpre(const LpDenseArgs &a, int n, int o) {
  const size_t i = (size_t)n * 32 + o;
  return a.Y[i] > 0.0f ? a.dY[i] : 0.0f;
}

// dX = dPre W^T; blockIdx.y selects 32 columns of X.
template <int KIND, bool BF16>
__global__ __launch_bounds__(kLpWG) void k_lp_dense_bwd(LpDenseArgs a) {
  constexpr int K = LpDims<KIND>::K;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int row0 = (blockIdx.x * 4 + wave) * 32;
  const int kcol = blockIdx.y * 32 + col;
  if (row0 >= a.N) return;
  const int r = row0 + col;
  const bool rv = r < a.N;
  lp_f16 acc;
  lp_zero(acc);
  if constexpr (BF16) {
    for (int o0 = 0; o0 < 32; o0 += 8) {
      lp_s4 av, bv;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int o = o0 + 4 * half + t;
        av[t] = lp_bf16(rv ? lp_dpre(a, r, o) : 0.0f);
        bv[t] = lp_bf16(a.W[kcol * 32 + o]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
  } else {
    for (int o0 = 0; o0 < 32; o0 += 2) {
      const int o = o0 + half;
      const float av = rv ? lp_dpre(a, r, o) : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, a.W[kcol * 32 + o], acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int q = 0; q < 16; q++) {
    const int row = row0 + lp_acc_row(q, half);
    if (row < a.N) a.dX[(size_t)row * K + kcol] = acc[q];
  }
}

// Weight and bias gradient partials of one workgroup (256 rows, 64 per
// wave): dW[k][o] = sum_n X[n][k] dPre[n][o], db[o] = sum_n dPre[n][o].
template <int KIND, bool BF16>
__global__ __launch_bounds__(kLpWG) void k_lp_wgrad(LpDenseArgs a) {
  constexpr int K = LpDims<KIND>::K, KR = LpDims<KIND>::KR, KT = (K + 31) / 32;
  __shared__ float red[4][KT * 1024];
  __shared__ float bred[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int nbase = blockIdx.x * 256 + wave * 64;
  lp_f16 acc[KT];
#pragma unroll
  for (int kt = 0; kt < KT; kt++) lp_zero(acc[kt]);
  float bsum = 0.0f;
  if constexpr (BF16) {
    for (int n0 = nbase; n0 < nbase + 64; n0 += 8) {
      lp_s4 bv;
      bool nv[4];
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int n = n0 + 4 * half + t;
        nv[t] = n < a.N;
        const float dp = nv[t] ? lp_dpre(a, n, col) : 0.0f;
        bsum += dp;
        bv[t] = lp_bf16(dp);
      }
#pragma unroll
      for (int kt = 0; kt < KT; kt++) {
        lp_s4 av;
        const int k = kt * 32 + col;
#pragma unroll
        for (int t = 0; t < 4; t++)
          av[t] = lp_bf16(nv[t] && k < KR ? lp_x<KIND>(a, n0 + 4 * half + t, k) : 0.0f);
        acc[kt] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc[kt], 0, 0, 0);
      }
    }
  } else {
    for (int n0 = nbase; n0 < nbase + 64; n0 += 2) {
      const int n = n0 + half;
      const bool nv = n < a.N;
      const float dp = nv ? lp_dpre(a, n, col) : 0.0f;
      bsum += dp;
#pragma unroll
      for (int kt = 0; kt < KT; kt++) {
        const int k = kt * 32 + col;
        const float av = nv && k < KR ? lp_x<KIND>(a, n, k) : 0.0f;
        acc[kt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, dp, acc[kt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int kt = 0; kt < KT; kt++)
#pragma unroll
    for (int q = 0; q < 16; q++) red[wave][kt * 1024 + lp_acc_row(q, half) * 32 + col] = acc[kt][q];
  bred[wave][lane] = bsum;
  __syncthreads();
  const int width = KR * 32 + 32;
  for (int idx = threadIdx.x; idx < width; idx += kLpWG) {
    float v = 0.0f;
    if (idx < KR * 32) {
      const int k = idx >> 5, o = idx & 31;
      const int li = (k >> 5) * 1024 + (k & 31) * 32 + o;
      v = red[0][li] + red[1][li] + red[2][li] + red[3][li];
    } else {
      const int o = idx - KR * 32;
      for (int w = 0; w < 4; w++) v += bred[w][o] + bred[w][o + 32];
    }
    a.part[(size_t)blockIdx.x * width + idx] = (double)v;
  }
}

__device__ inline double lp_softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }
__device__ inline double lp_sigmoid(double x) { return 0.5 * (1.0 + tanh(0.5 * x)); }

// gamma_i = he_i . w_hd + b_hd, gdiag = softplus(gamma); beta_p = z_p . w_p2 + b_p2,
// goff_p = beta_p mhat_p.
__global__ __launch_bounds__(kLpWG) void k_lp_heads_fwd(LpHeadArgs a) {
  const int ne = a.g.ne;
  const size_t idx = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  if (idx < (size_t)ne) {
    double s = a.b_hd[0];
    for (int o = 0; o < 32; o++) s += (double)a.he[idx * 32 + o] * a.w_hd[o];
    a.gam[idx] = s;
    a.gd[idx] = lp_softplus(s);
  } else if (idx < (size_t)5 * ne) {
    const size_t p = idx - ne;
    double s = a.b_p2[0];
    for (int o = 0; o < 32; o++) s += (double)a.z[p * 32 + o] * a.w_p2[o];
    a.goff[p] = s * a.g.mhat[p];
  }
}

// dL/dgamma = dL/dgdiag sigmoid(gamma), dL/dbeta = dL/dgoff mhat (in place);
// head parts of dL/dhe (initialises dhe) and dL/dz.
__global__ __launch_bounds__(kLpWG) void k_lp_heads_bwd(LpHeadArgs a) {
  const int ne = a.g.ne;
  const size_t idx = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  if (idx < (size_t)ne) {
    const double dg = a.ddiag[idx] * lp_sigmoid(a.gam[idx]);
    a.ddiag[idx] = dg;
    for (int o = 0; o < 32; o++) a.dhe[idx * 32 + o] = (float)(dg * a.w_hd[o]);
  } else if (idx < (size_t)5 * ne) {
    const size_t p = idx - ne;
    const double db = a.doff[p] * a.g.mhat[p];
    a.doff[p] = db;
    for (int o = 0; o < 32; o++) a.dz[p * 32 + o] = (float)(db * a.w_p2[o]);
  }
}

// part[wg][o] = sum_n s_n X[n][o], part[wg][32] = sum_n s_n over 256 rows.
__global__ __launch_bounds__(kLpWG) void k_lp_vgrad(LpVgradArgs a) {
  __shared__ double red[8][33];
  const int o = threadIdx.x & 31, grp = threadIdx.x >> 5;
  double acc = 0.0, ss = 0.0;
  for (int j = 0; j < 32; j++) {
    const int n = blockIdx.x * 256 + grp + 8 * j;
    if (n < a.N) {
      acc += a.s[n] * (double)a.X[(size_t)n * 32 + o];
      ss += a.s[n];
    }
  }
  red[grp][o] = acc;
  if (o == 0) red[grp][32] = ss;
  __syncthreads();
  if (threadIdx.x < 33) {
    double v = 0.0;
    for (int g = 0; g < 8; g++) v += red[g][threadIdx.x];
    a.part[(size_t)blockIdx.x * 33 + threadIdx.x] = v;
  }
}

// grad[i] += sum over groups of part[g][i], in group order.
__global__ __launch_bounds__(kLpWG) void k_lp_wreduce(const double *part, int groups, int width,
                                                      double *grad) {
  const int i = blockIdx.x * kLpWG + threadIdx.x;
  if (i >= width) return;
  double v = 0.0;
  for (int g = 0; g < groups; g++) v += part[(size_t)g * width + i];
  grad[i] += v;
}

// out = Ghat in (transpose = 0) or Ghat^T in (transpose = 1), probes in
// [row][P]; with res: res = out - z and loss partials sum res^2 / |z_p|^2.
__global__ __launch_bounds__(kLpWG) void k_lp_probe_G(LpProbeArgs a) {
  __shared__ double red[kLpWG];
  const int P = a.P;
  const size_t idx = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  double l = 0.0;
  if (idx < (size_t)a.g.ne * P) {
    const int i = (int)(idx / P), p = (int)(idx % P);
    double v = a.gd[i] * a.in[idx];
    for (int s = 0; s < 4; s++) {
      const int q = 4 * i + s;
      const double gv = a.transpose ? a.goff[a.g.tpos[q]] : a.goff[q];
      v += gv * a.in[(size_t)a.g.pj[q] * P + p];
    }
    a.out[idx] = v;
    if (a.res) {
      const double r = v - a.z[idx];
      a.res[idx] = r;
      l = r * r * a.zinv[p];
    }
  }
  if (!a.res) return;
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = kLpWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = red[0];
}

// out = Mhat in
__global__ __launch_bounds__(kLpWG) void k_lp_probe_M(LpProbeArgs a) {
  const int P = a.P;
  const size_t idx = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  if (idx >= (size_t)a.g.ne * P) return;
  const int i = (int)(idx / P), p = (int)(idx % P);
  double v = 0.0;
  for (int j = 0; j < 5; j++) v += a.g.mval[5 * i + j] * a.in[(size_t)a.g.mcol[5 * i + j] * P + p];
  a.out[idx] = v;
}

// dL/dGhat_ij = (2/P) sum_p (w_i res_j + u_i z_j) / |z_p|^2 on the pattern.
__global__ __launch_bounds__(kLpWG) void k_lp_ghat_grad(LpGhatGradArgs a) {
  const int i = blockIdx.x * kLpWG + threadIdx.x;
  if (i >= a.g.ne) return;
  const int P = a.P;
  const double sc = 2.0 / P;
  double dd = 0.0;
  for (int p = 0; p < P; p++) {
    const size_t ii = (size_t)i * P + p;
    dd += sc * a.zinv[p] * (a.w[ii] * a.res[ii] + a.u[ii] * a.z[ii]);
  }
  a.ddiag[i] = dd;
  for (int s = 0; s < 4; s++) {
    const int q = 4 * i + s, j = a.g.pj[q];
    double v = 0.0;
    for (int p = 0; p < P; p++) {
      const size_t ii = (size_t)i * P + p, jj = (size_t)j * P + p;
      v += sc * a.zinv[p] * (a.w[ii] * a.res[jj] + a.u[ii] * a.z[jj]);
    }
    a.doff[q] = v;
  }
}

// Gradients of gathered inputs back to the activations they came from, as
// gathers over the inverse adjacency (deterministic, no atomics).
__global__ __launch_bounds__(kLpWG) void k_lp_scatter(LpScatterArgs a) {
  const int ne = a.g.ne, nc = a.g.nc;
  const size_t idx = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  const int o = (int)(idx & 31);
  const size_t row = idx >> 5;
  if (a.mode == LP_SC_PAIR) {
    if (row < (size_t)ne) {
      const int e = (int)row;
      float v = a.dhe[row * 32 + o];
      for (int s = 0; s < 4; s++) {
        v += a.dxp[(size_t)(4 * e + s) * 96 + o];
        v += a.dxp[(size_t)a.g.tpos[4 * e + s] * 96 + 32 + o];
      }
      a.dhe[row * 32 + o] = v;
    } else if (row < (size_t)ne + nc) {
      const size_t c = row - ne;
      float v = 0.0f;
      for (int t = 0; t < 6; t++) v += a.dxp[(size_t)a.g.revc[6 * c + t] * 96 + 64 + o];
      a.dhc[c * 32 + o] = v;
    }
  } else if (a.mode == LP_SC_CELLS_FROM_EDGES) {
    if (row < (size_t)nc) {
      const int32_t *e = a.g.ce + 3 * row;
      a.dhc[row * 32 + o] += 0.5f * (a.dxe[(size_t)e[0] * 64 + 32 + o] + a.dxe[(size_t)e[1] * 64 + 32 + o] +
                                     a.dxe[(size_t)e[2] * 64 + 32 + o]);
    }
  } else if (a.mode == LP_SC_EDGES) {
    if (row < (size_t)ne) {
      const int32_t *c = a.g.ec + 2 * row;
      a.dhe[row * 32 + o] = a.dxe[row * 64 + o] + (a.dxc[(size_t)c[0] * 64 + 32 + o] +
                                                   a.dxc[(size_t)c[1] * 64 + 32 + o]) * (1.0f / 3.0f);
    }
  } else {  // LP_SC_CELLS_DIRECT
    if (row < (size_t)nc) a.dhc[row * 32 + o] = a.dxc[row * 64 + o];
  }
}

__global__ __launch_bounds__(kLpWG) void k_lp_adam(LpAdamArgs a) {
  const int i = blockIdx.x * kLpWG + threadIdx.x;
  if (i >= a.n) return;
  const double g = a.grad[i] * a.gscale;
  const double m = a.b1 * a.m[i] + (1.0 - a.b1) * g;
  const double v = a.b2 * a.v[i] + (1.0 - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.theta[i] = (float)((double)a.theta[i] - a.lr * (m / a.c1) / (sqrt(v / a.c2) + a.eps));
}

// Rademacher probes from a counter-based hash (SplitMix64 finaliser).
__global__ __launch_bounds__(kLpWG) void k_lp_rademacher(double *z, size_t n, uint64_t seed) {
  const size_t i = (size_t)blockIdx.x * kLpWG + threadIdx.x;
  if (i >= n) return;
  uint64_t x = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  z[i] = (x >> 63) ? 1.0 : -1.0;
}

__global__ __launch_bounds__(kLpWG) void k_lp_loss_reduce(const double *part, int groups, double *out) {
  __shared__ double red[kLpWG];
  double v = 0.0;
  for (int g = threadIdx.x; g < groups; g += kLpWG) v += part[g];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kLpWG / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

int blocks_for(size_t n) { return (int)((n + kLpWG - 1) / kLpWG); }

template <int KIND>
void fwd_k(bool bf16, const LpDenseArgs &a, hipStream_t s) {
  const dim3 grid((a.N + 127) / 128);
  if (bf16)
    hipLaunchKernelGGL((k_lp_dense_fwd<KIND, true>), grid, dim3(kLpWG), 0, s, a);
  else
    hipLaunchKernelGGL((k_lp_dense_fwd<KIND, false>), grid, dim3(kLpWG), 0, s, a);
}
template <int KIND>
void bwd_k(bool bf16, const LpDenseArgs &a, hipStream_t s) {
  const dim3 grid((a.N + 127) / 128, LpDims<KIND>::K / 32);
  if (bf16)
    hipLaunchKernelGGL((k_lp_dense_bwd<KIND, true>), grid, dim3(kLpWG), 0, s, a);
  else
    hipLaunchKernelGGL((k_lp_dense_bwd<KIND, false>), grid, dim3(kLpWG), 0, s, a);
}
template <int KIND>
void wgrad_k(bool bf16, const LpDenseArgs &a, hipStream_t s) {
  const dim3 grid(lp_wgrad_groups(a.N));
  if (bf16)
    hipLaunchKernelGGL((k_lp_wgrad<KIND, true>), grid, dim3(kLpWG), 0, s, a);
  else
    hipLaunchKernelGGL((k_lp_wgrad<KIND, false>), grid, dim3(kLpWG), 0, s, a);
}

}  // namespace

int lp_in_dim(int kind) {
  switch (kind) {
    case LP_ENC_E: return kLpFE;
    case LP_ENC_C: return kLpFC;
    case LP_PAIR: return 96;
    default: return 64;
  }
}

int lp_rows(const LpGraphDev &g, int kind) {
  switch (kind) {
    case LP_ENC_E:
    case LP_EDGE: return g.ne;
    case LP_PAIR: return 4 * g.ne;
    default: return g.nc;
  }
}

int lp_wgrad_groups(int N) { return (N + 255) / 256; }
int lp_probe_groups(int ne, int P) { return blocks_for((size_t)ne * P); }

void launch_lp_dense_fwd(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s) {
  switch (kind) {
    case LP_ENC_E: fwd_k<LP_ENC_E>(bf16, a, s); break;
    case LP_ENC_C: fwd_k<LP_ENC_C>(bf16, a, s); break;
    case LP_CELL: fwd_k<LP_CELL>(bf16, a, s); break;
    case LP_EDGE: fwd_k<LP_EDGE>(bf16, a, s); break;
    default: fwd_k<LP_PAIR>(bf16, a, s); break;
  }
}

void launch_lp_dense_bwd(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s) {
  switch (kind) {
    case LP_CELL: bwd_k<LP_CELL>(bf16, a, s); break;
    case LP_EDGE: bwd_k<LP_EDGE>(bf16, a, s); break;
    case LP_PAIR: bwd_k<LP_PAIR>(bf16, a, s); break;
    default: throw Error(PA_EINVAL, "encoder inputs have no gradient");
  }
}

void launch_lp_wgrad(int kind, bool bf16, const LpDenseArgs &a, hipStream_t s) {
  switch (kind) {
    case LP_ENC_E: wgrad_k<LP_ENC_E>(bf16, a, s); break;
    case LP_ENC_C: wgrad_k<LP_ENC_C>(bf16, a, s); break;
    case LP_CELL: wgrad_k<LP_CELL>(bf16, a, s); break;
    case LP_EDGE: wgrad_k<LP_EDGE>(bf16, a, s); break;
    default: wgrad_k<LP_PAIR>(bf16, a, s); break;
  }
}

void launch_lp_heads_fwd(const LpHeadArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_heads_fwd, dim3(blocks_for((size_t)5 * a.g.ne)), dim3(kLpWG), 0, s, a);
}
void launch_lp_heads_bwd(const LpHeadArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_heads_bwd, dim3(blocks_for((size_t)5 * a.g.ne)), dim3(kLpWG), 0, s, a);
}
void launch_lp_vgrad(const LpVgradArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_vgrad, dim3(lp_wgrad_groups(a.N)), dim3(kLpWG), 0, s, a);
}
void launch_lp_wreduce(const double *part, int groups, int width, double *grad, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_wreduce, dim3(blocks_for(width)), dim3(kLpWG), 0, s, part, groups, width, grad);
}
void launch_lp_probe_G(const LpProbeArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_probe_G, dim3(lp_probe_groups(a.g.ne, a.P)), dim3(kLpWG), 0, s, a);
}
void launch_lp_probe_M(const LpProbeArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_probe_M, dim3(lp_probe_groups(a.g.ne, a.P)), dim3(kLpWG), 0, s, a);
}
void launch_lp_ghat_grad(const LpGhatGradArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_ghat_grad, dim3(blocks_for(a.g.ne)), dim3(kLpWG), 0, s, a);
}
void launch_lp_scatter(const LpScatterArgs &a, hipStream_t s) {
  const size_t rows = a.mode == LP_SC_PAIR ? (size_t)a.g.ne + a.g.nc
                      : a.mode == LP_SC_EDGES ? (size_t)a.g.ne
                                              : (size_t)a.g.nc;
  hipLaunchKernelGGL(k_lp_scatter, dim3(blocks_for(rows * 32)), dim3(kLpWG), 0, s, a);
}
void launch_lp_adam(const LpAdamArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_adam, dim3(blocks_for(a.n)), dim3(kLpWG), 0, s, a);
}
void launch_lp_rademacher(double *z, int ne, int P, uint64_t seed, hipStream_t s) {
  const size_t n = (size_t)ne * P;
  hipLaunchKernelGGL(k_lp_rademacher, dim3(blocks_for(n)), dim3(kLpWG), 0, s, z, n, seed);
}
void launch_lp_loss_reduce(const double *part, int groups, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_loss_reduce, dim3(1), dim3(kLpWG), 0, s, part, groups, out);
}

}  // namespace pa
