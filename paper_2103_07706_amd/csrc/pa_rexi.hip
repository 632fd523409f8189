// HIP kernels of the rational (REXI) exponential of libpa for gfx950.
//
// The P independent shifted systems of a call (times the members) are the
// complex columns of one block, row-major [row][Bc] of double2, so that a
// gathered ELL neighbour row is one contiguous run of 16-byte values.  A
// launch covers a tile of CT = min(Bc, 64) columns (blockIdx.y) and an
// XCD-aware grid-stride range of velocity rows (as the real block kernels:
// each XCD takes one contiguous slice of rows, so ELL neighbours meet in its
// L2).  Every column runs its own BiCGStab (left Jacobi preconditioning,
// Hermitian inner products, a counter-hash shadow residual); converged
// columns freeze.  Column sums go through per-workgroup partials with plain
// stores and a finalize kernel per reduction point (one workgroup per column,
// fixed summation order), so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include "pa_rexi.h"

namespace pa {

namespace {
constexpr int kRWG = 256;

struct RLane {
  int ct, rw, col, tile, row0, rstride, rend, lane, wave;
};

__device__ inline RLane rlane(int Bc, int nrows) {
  RLane L;
  L.ct = Bc < 64 ? Bc : 64;
  L.rw = 64 / L.ct;
  L.lane = threadIdx.x & 63;
  L.wave = threadIdx.x >> 6;
  L.tile = blockIdx.y;
  L.col = L.tile * L.ct + (L.lane % L.ct);
  const int per = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
  const int slice = (nrows + 7) >> 3;
  const int rpp = (kRWG / 64) * L.rw;
  L.rend = min(nrows, (xcd + 1) * slice);
  L.row0 = xcd * slice + w * rpp + L.wave * L.rw + L.lane / L.ct;
  L.rstride = per * rpp;
  return L;
}

// One row per wave (UNI: blocks of 64 or more columns, lane = column of a
// 64-column tile): the row number is wave-uniform, so the row's operator
// entries load through the scalar unit instead of once per lane.
__device__ inline RLane rlane_uni(int nrows) {
  RLane L;
  L.ct = 64;
  L.rw = 1;
  L.lane = threadIdx.x & 63;
  L.wave = threadIdx.x >> 6;
  L.tile = blockIdx.y;
  L.col = L.tile * 64 + L.lane;
  const int per = gridDim.x >> 3;
  const int xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
  const int slice = (nrows + 7) >> 3;
  const int rpp = kRWG / 64;
  L.rend = min(nrows, (xcd + 1) * slice);
  L.row0 = xcd * slice + w * rpp + L.wave;
  L.rstride = per * rpp;
  return L;
}
template <bool UNI>
__device__ inline RLane rlane_t(int Bc, int nrows) {
  return UNI ? rlane_uni(nrows) : rlane(Bc, nrows);
}

// Row-table loads: through the constant address space (scalar loads) when
// the row is wave-uniform.
template <bool UNI, typename T>
__device__ inline T rld(const T *p, size_t i) {
  if constexpr (UNI)
    return ((const __attribute__((address_space(4))) T *)p)[i];
  else
    return p[i];
}
template <bool UNI>
__device__ inline uint2 rld(const uint2 *p, size_t i) {
  if constexpr (UNI) {
    const unsigned long long v = ((const __attribute__((address_space(4))) unsigned long long *)p)[i];
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
  } else {
    return p[i];
  }
}
template <bool UNI>
__device__ inline int urow(int e) {
  return UNI ? __builtin_amdgcn_readfirstlane(e) : e;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// a / b through the hardware reciprocal of |b|^2 and two Newton steps (full
// FP64 accuracy from its estimate; |b|^2 is a positive normal number here:
// a diagonal of a shifted system)
__device__ inline double2 cdiv(double2 a, double2 b) {
  const double n = b.x * b.x + b.y * b.y;
  double inv = __builtin_amdgcn_rcp(n);
  inv = fma(inv, fma(-n, inv, 1.0), inv);
  inv = fma(inv, fma(-n, inv, 1.0), inv);
  return make_double2((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);
}
// a / b with IEEE division (the scalars of the iteration, of any magnitude)
__device__ inline double2 cdiv_ieee(double2 a, double2 b) {
  const double n = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / n, (a.y * b.x - a.x * b.y) / n);
}
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// conj(a) b
__device__ inline double2 cdotc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Shadow residual of BiCGStab: a 32-bit counter hash (multiply-xorshift
// rounds) of the row, the column and the seed, two 16-bit halves mapped to
// [-1, 1).
__device__ inline double2 shadow(uint32_t seed, int e, int col) {
  uint32_t h = (uint32_t)e * 0x9E3779B1u ^ ((uint32_t)col + 1u) * 0x85EBCA77u ^ seed;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  const double sc = 1.0 / 32768.0;
  return make_double2((double)(h & 0xFFFFu) * sc - 1.0, (double)(h >> 16) * sc - 1.0);
}

// Per-workgroup column sums of NQ quantities into part[wg][q][Bc].
template <int NQ>
__device__ void rexi_partials(const RLane &L, double (&v)[NQ], double *part, int Bc) {
  __shared__ double red[NQ][kRWG / 64][64];
  for (int q = 0; q < NQ; q++) {
    double s = v[q];
    for (int off = 32; off >= L.ct; off >>= 1) s += __shfl_xor(s, off);
    if (L.lane < L.ct) red[q][L.wave][L.lane] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NQ * L.ct; idx += kRWG) {
    const int q = idx / L.ct, c = idx % L.ct;
    if (L.tile * L.ct + c >= Bc) continue;  // lanes past the block (one-row-a-wave form)
    double s = 0;
    for (int w = 0; w < kRWG / 64; w++) s += red[q][w][c];
    part[((size_t)blockIdx.x * NQ + q) * Bc + L.tile * L.ct + c] = s;
  }
}

// Sum of quantity q of column col over nwg workgroup partials (one
// workgroup per column; fixed order).  Result valid in thread 0.
__device__ double col_sum(const double *part, int nq, int q, int Bc, int col, int nwg) {
  __shared__ double red[kRWG];
  double s = 0;
  for (int w = threadIdx.x; w < nwg; w += kRWG) s += part[((size_t)w * nq + q) * Bc + col];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kRWG / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Velocity part of the right-hand side of column col at edge e:
// f = M_u U_u + q (U_eta(c0) - U_eta(c1)).
template <bool UNI>
__device__ inline double2 rhs_u(const RexiArgs &a, int e, int col, double2 q) {
  const DevOps &o = a.ops;
  const int c0 = rld<UNI>(o.ecell, 2 * e), c1 = rld<UNI>(o.ecell, 2 * e + 1);
  if (a.src.real_blk) {
    const int Bm = a.src.Bm, mem = col / a.P;
    const double *U = a.src.real_blk;
    double mu = 0.0;
#pragma unroll
    for (int k = 0; k < 5; k++)
      mu = fma(rld<UNI>(o.mass, 5 * e + k), U[(size_t)rld<UNI>(o.ell_col, 5 * e + k) * Bm + mem], mu);
    const double de = U[(size_t)(o.ne + c0) * Bm + mem] - U[(size_t)(o.ne + c1) * Bm + mem];
    return make_double2(mu + q.x * de, q.y * de);
  }
  const double2 *Z = a.src.cplx_blk;
  const int Bc = a.Bc;
  double2 mu = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const double m = rld<UNI>(o.mass, 5 * e + k);
    const double2 z = Z[(size_t)rld<UNI>(o.ell_col, 5 * e + k) * Bc + col];
    mu.x = fma(m, z.x, mu.x);
    mu.y = fma(m, z.y, mu.y);
  }
  const double2 de = csub(Z[(size_t)(o.ne + c0) * Bc + col], Z[(size_t)(o.ne + c1) * Bc + col]);
  return cadd(mu, cmul(q, de));
}

// (S z)_e for column col, S = a M + b F + c G (b = -i binv), with z read by
// the gather g(row); also the diagonal of S at e.
template <bool UNI, class Gz>
__device__ inline double2 schur_row(const RexiArgs &a, int e, double2 ca, double2 cc, Gz g, double2 &diag) {
  const DevOps &o = a.ops;
  double2 mz = make_double2(0.0, 0.0), fz = mz, gz = mz;
#pragma unroll
  for (int k = 0; k < 5; k++) {
    const int j = rld<UNI>(o.ell_col, 5 * e + k);
    const double2 z = g(j);
    const double m = rld<UNI>(o.mass, 5 * e + k), f = rld<UNI>(o.cor, 5 * e + k);
    const double gg = rld<UNI>(o.graddiv, 5 * e + k);
    mz.x = fma(m, z.x, mz.x);
    mz.y = fma(m, z.y, mz.y);
    fz.x = fma(f, z.x, fz.x);
    fz.y = fma(f, z.y, fz.y);
    gz.x = fma(gg, z.x, gz.x);
    gz.y = fma(gg, z.y, gz.y);
  }
  diag = cadd(cscale(rld<UNI>(o.mass, 5 * e), ca), cscale(rld<UNI>(o.graddiv, 5 * e), cc));
  // b F z = -i binv F z = binv (Im Fz, -Re Fz)
  return cadd(cadd(cmul(ca, mz), cmul(cc, gz)), make_double2(a.binv * fz.y, -a.binv * fz.x));
}

// ---------------------------------------------------------------- kernels
// Start (mode 0: x = 0, residual f) or check-and-restart (mode 1: residual
// f - S x) of every valid column: r = D^-1 res, p = r.  Partials: |res|^2,
// |r|^2, (r~, r).
template <bool UNI>
__global__ __launch_bounds__(kRWG) void k_rexi_init(RexiArgs a, double2 *p_out) {
  const RLane L = rlane_t<UNI>(a.Bc, a.ops.ne);
  const int col = L.col;
  const bool on = col < a.ncols;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (on) {
    const double2 ca = a.co.a[col], cc = a.co.c[col], cq = a.co.q[col];
    for (int base = L.row0; base < L.rend; base += L.rstride) {
      const int e = urow<UNI>(base);
      const size_t ie = (size_t)e * a.Bc + col;
      double2 res = rhs_u<UNI>(a, e, col, cq);
      double2 d;
      if (a.mode == 1) {
        const double2 *x = a.x;
        const int Bc = a.Bc;
        const double2 sx = schur_row<UNI>(a, e, ca, cc, [&](int j) { return x[(size_t)j * Bc + col]; }, d);
        res = csub(res, sx);
      } else {
        d = cadd(cscale(rld<UNI>(a.ops.mass, 5 * e), ca), cscale(rld<UNI>(a.ops.graddiv, 5 * e), cc));
        a.x[ie] = make_double2(0.0, 0.0);
      }
      if (a.lp) {  // k_rexi_lp forms r = P res / X and the partials
        a.w[ie] = res;
        continue;
      }
      const double2 r = cdiv(res, d);
      a.r[ie] = r;
      p_out[ie] = r;
      v[0] += cabs2(res);
      v[1] += cabs2(r);
      const double2 rr = cdotc(shadow(a.seed, e, col), r);
      v[2] += rr.x;
      v[3] += rr.y;
    }
  }
  rexi_partials<4>(L, v, a.part, a.Bc);
}

__global__ __launch_bounds__(kRWG) void k_rexi_fin_init(RexiArgs a, int nwg) {
  const int col = blockIdx.x;
  const double res2 = col_sum(a.part, 4, 0, a.Bc, col, nwg);
  const double r2 = col_sum(a.part, 4, 1, a.Bc, col, nwg);
  const double rre = col_sum(a.part, 4, 2, a.Bc, col, nwg);
  const double rim = col_sum(a.part, 4, 3, a.Bc, col, nwg);
  if (threadIdx.x != 0) return;
  RexiState st = a.st;
  if (col >= a.ncols) {
    st.active[col] = 0;
    return;
  }
  if (a.mode == 0) {
    st.ff[col] = res2;
    st.bb[col] = r2;
    st.res2[col] = res2;
    st.tau2[col] = a.rtol2;
    st.rho[col] = make_double2(rre, rim);
    st.active[col] = res2 > 0.0 ? 1 : 0;
    st.iters[col] = 0;
    st.fresh[col] = 1;
    st.restarts[col] = 0;
    return;
  }
  st.res2[col] = res2;
  if (st.ff[col] == 0.0 || res2 <= a.rtol2 * st.ff[col]) {
    st.active[col] = 0;
    return;
  }
  if (st.iters[col] >= a.maxit) {  // no iterations left to restart with
    st.active[col] = 0;
    atomicAdd(st.fail, 1);
    return;
  }
  // restart from x with a target tightened by the miss of the true residual
  st.tau2[col] = st.tau2[col] * fmin(0.25, 0.25 * a.rtol2 * st.ff[col] / res2);
  st.rho[col] = make_double2(rre, rim);
  st.active[col] = 1;
  st.fresh[col] = 1;
  st.restarts[col] += 1;
}

// p' = r + beta (p - omega v) (p' = p on a fresh start): a streaming pass,
// so that the operator application gathers one vector only.
__global__ __launch_bounds__(kRWG) void k_rexi_p(RexiArgs a, const double2 *p_in, const double2 *v_in,
                                                   double2 *p_out) {
  const RLane L = rlane(a.Bc, a.ops.ne);
  const int col = L.col, Bc = a.Bc;
  if (col >= a.ncols || !a.st.active[col]) return;
  const bool fresh = a.st.fresh[col] != 0;
  const double2 beta = a.st.beta[col], omega = a.st.omega[col];
  for (int e = L.row0; e < L.rend; e += L.rstride) {
    const size_t ie = (size_t)e * Bc + col;
    p_out[ie] = fresh ? p_in[ie] : cadd(a.r[ie], cmul(beta, csub(p_in[ie], cmul(omega, v_in[ie]))));
  }
}

// v' = D^-1 S p'.  Partials: (r~, v').
template <bool UNI>
__global__ __launch_bounds__(kRWG) void k_rexi_sv(RexiArgs a, const double2 *p_in, double2 *v_out) {
  const RLane L = rlane_t<UNI>(a.Bc, a.ops.ne);
  const int col = L.col, Bc = a.Bc;
  const bool on = col < a.ncols && a.st.active[col];
  double v[2] = {0.0, 0.0};
  if (on) {
    const double2 ca = a.co.a[col], cc = a.co.c[col];
    for (int base = L.row0; base < L.rend; base += L.rstride) {
      const int e = urow<UNI>(base);
      double2 d;
      const double2 sp = schur_row<UNI>(a, e, ca, cc, [&](int j) { return p_in[(size_t)j * Bc + col]; }, d);
      if (a.lp) {
        a.w[(size_t)e * Bc + col] = sp;
        continue;
      }
      const double2 vv = cdiv(sp, d);
      v_out[(size_t)e * Bc + col] = vv;
      const double2 rv = cdotc(shadow(a.seed, e, col), vv);
      v[0] += rv.x;
      v[1] += rv.y;
    }
  }
  rexi_partials<2>(L, v, a.part, a.Bc);
}

__global__ __launch_bounds__(kRWG) void k_rexi_fin_v(RexiArgs a, int nwg) {
  const int col = blockIdx.x;
  const double re = col_sum(a.part, 2, 0, a.Bc, col, nwg);
  const double im = col_sum(a.part, 2, 1, a.Bc, col, nwg);
  if (threadIdx.x != 0 || col >= a.ncols || !a.st.active[col]) return;
  const double2 rv = make_double2(re, im);
  if (cabs2(rv) == 0.0) {  // breakdown: leave the column to the residual check
    a.st.alpha[col] = make_double2(0.0, 0.0);
    a.st.active[col] = 0;
    return;
  }
  a.st.alpha[col] = cdiv_ieee(a.st.rho[col], rv);
}

// s = r - alpha v, t = D^-1 S s.  Partials: (t, s), |t|^2.
template <bool UNI>
__global__ __launch_bounds__(kRWG) void k_rexi_t(RexiArgs a, const double2 *v_in) {
  const RLane L = rlane_t<UNI>(a.Bc, a.ops.ne);
  const int col = L.col, Bc = a.Bc;
  const bool on = col < a.ncols && a.st.active[col];
  double v[3] = {0.0, 0.0, 0.0};
  if (on) {
    const double2 ca = a.co.a[col], cc = a.co.c[col];
    const double2 alpha = a.st.alpha[col];
    const double2 *r = a.r;
    auto snew = [&](int j) {
      const size_t ij = (size_t)j * Bc + col;
      return csub(r[ij], cmul(alpha, v_in[ij]));
    };
    for (int base = L.row0; base < L.rend; base += L.rstride) {
      const int e = urow<UNI>(base);
      const size_t ie = (size_t)e * Bc + col;
      double2 d;
      const double2 ss = snew(e);
      const double2 ws = schur_row<UNI>(a, e, ca, cc, snew, d);
      if (a.lp) {
        a.s[ie] = ss;
        a.w[ie] = ws;
        continue;
      }
      const double2 tt = cdiv(ws, d);
      a.s[ie] = ss;
      a.t[ie] = tt;
      const double2 ts = cdotc(tt, ss);
      v[0] += ts.x;
      v[1] += ts.y;
      v[2] += cabs2(tt);
    }
  }
  rexi_partials<3>(L, v, a.part, a.Bc);
}

__global__ __launch_bounds__(kRWG) void k_rexi_fin_t(RexiArgs a, int nwg) {
  const int col = blockIdx.x;
  const double re = col_sum(a.part, 3, 0, a.Bc, col, nwg);
  const double im = col_sum(a.part, 3, 1, a.Bc, col, nwg);
  const double tt = col_sum(a.part, 3, 2, a.Bc, col, nwg);
  if (threadIdx.x != 0 || col >= a.ncols || !a.st.active[col]) return;
  a.st.omega[col] = tt > 0.0 ? make_double2(re / tt, im / tt) : make_double2(0.0, 0.0);
}

// x += alpha p + omega s, r = s - omega t.  Partials: (r~, r), |r|^2.
__global__ __launch_bounds__(kRWG) void k_rexi_x(RexiArgs a, const double2 *p_in) {
  const RLane L = rlane(a.Bc, a.ops.ne);
  const int col = L.col, Bc = a.Bc;
  const bool on = col < a.ncols && a.st.active[col];
  double v[3] = {0.0, 0.0, 0.0};
  if (on) {
    const double2 alpha = a.st.alpha[col], omega = a.st.omega[col];
    for (int e = L.row0; e < L.rend; e += L.rstride) {
      const size_t ie = (size_t)e * Bc + col;
      const double2 ss = a.s[ie];
      a.x[ie] = cadd(a.x[ie], cadd(cmul(alpha, p_in[ie]), cmul(omega, ss)));
      const double2 rn = csub(ss, cmul(omega, a.t[ie]));
      a.r[ie] = rn;
      const double2 rr = cdotc(shadow(a.seed, e, col), rn);
      v[0] += rr.x;
      v[1] += rr.y;
      v[2] += cabs2(rn);
    }
  }
  rexi_partials<3>(L, v, a.part, a.Bc);
}

__global__ __launch_bounds__(kRWG) void k_rexi_fin_x(RexiArgs a, int nwg) {
  const int col = blockIdx.x;
  const double re = col_sum(a.part, 3, 0, a.Bc, col, nwg);
  const double im = col_sum(a.part, 3, 1, a.Bc, col, nwg);
  const double r2 = col_sum(a.part, 3, 2, a.Bc, col, nwg);
  if (threadIdx.x != 0 || col >= a.ncols || !a.st.active[col]) return;
  RexiState st = a.st;
  const int it = ++st.iters[col];
  st.fresh[col] = 0;
  const double2 rho_new = make_double2(re, im), omega = st.omega[col];
  if (r2 <= st.tau2[col] * st.bb[col]) {  // to the true-residual check
    st.active[col] = 0;
    return;
  }
  if (cabs2(omega) == 0.0 || cabs2(rho_new) == 0.0) {  // breakdown: check and restart
    st.active[col] = 0;
    return;
  }
  if (it >= a.maxit) {
    st.active[col] = 0;
    atomicAdd(st.fail, 1);
    return;
  }
  st.beta[col] = cmul(cdiv_ieee(rho_new, st.rho[col]), cdiv_ieee(st.alpha[col], omega));
  st.rho[col] = rho_new;
}

// Learned left preconditioner: y = P w / X (P real, FP32 values, FP64
// arithmetic), then the partials the Jacobi kernels would have formed.
template <bool UNI>
__global__ __launch_bounds__(kRWG) void k_rexi_lp(RexiArgs a, int kind, double2 *y_out, double2 *p_out) {
  const RLane L = rlane_t<UNI>(a.Bc, a.ops.ne);
  const int col = L.col, Bc = a.Bc, ne = a.ops.ne;
  const bool on = col < a.ncols && (kind == 0 || a.st.active[col]);
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (on) {
    const double2 xinv = a.co.xinv[col];
    for (int base = L.row0; base < L.rend; base += L.rstride) {
      const int e = urow<UNI>(base);
      const size_t ie = (size_t)e * Bc + col;
      double2 z = make_double2(0.0, 0.0);
      for (int k = 0; k < a.lpw; k++) {
        const uint2 q = rld<UNI>(a.lp, (size_t)k * ne + e);
        const double pv = (double)__uint_as_float(q.y);
        const double2 wv = a.w[(size_t)q.x * Bc + col];
        z.x = fma(pv, wv.x, z.x);
        z.y = fma(pv, wv.y, z.y);
      }
      const double2 y = cmul(xinv, z);
      y_out[ie] = y;
      const double2 sh = cdotc(shadow(a.seed, e, col), y);
      if (kind == 0) {
        p_out[ie] = y;
        v[0] += cabs2(a.w[ie]);
        v[1] += cabs2(y);
        v[2] += sh.x;
        v[3] += sh.y;
      } else if (kind == 1) {
        v[0] += sh.x;
        v[1] += sh.y;
      } else {
        const double2 ts = cdotc(y, a.s[ie]);
        v[0] += ts.x;
        v[1] += ts.y;
        v[2] += cabs2(y);
      }
    }
  }
  if (kind == 0) {
    rexi_partials<4>(L, v, a.part, a.Bc);
  } else if (kind == 1) {
    double u[2] = {v[0], v[1]};
    rexi_partials<2>(L, u, a.part, a.Bc);
  } else {
    double u[3] = {v[0], v[1], v[2]};
    rexi_partials<3>(L, u, a.part, a.Bc);
  }
}

// Depth rows: y_eta = xinv src_eta + h (D y_u) / |c|.
__global__ __launch_bounds__(kRWG) void k_rexi_eta(RexiEtaArgs a) {
  const RLane L = rlane(a.Bc, a.ops.nc);
  const int col = L.col, Bc = a.Bc;
  if (col >= Bc) return;
  const DevOps &o = a.ops;
  const bool on = col < a.ncols;
  const double2 xinv = on ? a.co.xinv[col] : make_double2(0.0, 0.0);
  const double2 h = on ? a.co.h[col] : make_double2(0.0, 0.0);
  for (int t = L.row0; t < L.rend; t += L.rstride) {
    const size_t it = (size_t)t * Bc + col;
    if (!on) {
      a.yeta[it] = make_double2(0.0, 0.0);
      continue;
    }
    double2 div = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 3; j++) {
      const double sg = (double)o.csgn[3 * t + j];
      const double2 y = a.yu[(size_t)o.cedge[3 * t + j] * Bc + col];
      div.x = fma(sg, y.x, div.x);
      div.y = fma(sg, y.y, div.y);
    }
    double2 src;
    if (a.src.real_blk)
      src = make_double2(a.src.real_blk[(size_t)(o.ne + t) * a.src.Bm + col / a.P], 0.0);
    else
      src = a.src.cplx_blk[(size_t)(o.ne + t) * Bc + col];
    a.yeta[it] = cadd(cmul(xinv, src), cscale(o.inv_area[t], cmul(h, div)));
  }
}

__global__ __launch_bounds__(kRWG) void k_rexi_combine(RexiCombineArgs a) {
  const int Bo = a.members * a.Go, So = a.ostride;
  const size_t total = (size_t)a.n * So;
  for (size_t i = (size_t)blockIdx.x * kRWG + threadIdx.x; i < total; i += (size_t)gridDim.x * kRWG) {
    const int row = (int)(i / So), oc = (int)(i % So);
    const int mem = oc / a.Go, m = oc % a.Go;
    double acc = 0.0;
    if (oc < Bo && m < a.Mo) {
      const double2 *C = a.C + ((size_t)(a.per_member ? mem : 0) * a.Go + m) * a.P;
      const double2 *Y = a.Y + (size_t)row * a.Bc + (size_t)mem * a.P;
      for (int j = 0; j < a.P; j++) {
        const double2 c = C[j], y = Y[j];
        acc = fma(c.x, y.x, acc);
        acc = fma(-c.y, y.y, acc);
      }
    }
    a.out[i] = acc;
  }
}

__global__ __launch_bounds__(kRWG) void k_rexi_back(RexiBackArgs a) {
  const size_t total = (size_t)a.n * a.Bc;
  const int Bi = a.istride;
  for (size_t i = (size_t)blockIdx.x * kRWG + threadIdx.x; i < total; i += (size_t)gridDim.x * kRWG) {
    const int row = (int)(i / a.Bc), col = (int)(i % a.Bc);
    double2 z = make_double2(0.0, 0.0);
    if (col < a.members * a.P) {
      const int mem = col / a.P, j = col % a.P;
      const double *Yn = a.Yn + (size_t)row * Bi + (size_t)mem * a.Gi;
      for (int m = 0; m < a.Mi; m++) {
        const double2 c = a.C[(size_t)m * a.P + j];
        const double y = Yn[m];
        z.x = fma(c.x, y, z.x);
        z.y = fma(c.y, y, z.y);
      }
    }
    a.Z[i] = z;
  }
}
}  // namespace

// ------------------------------------------------------------ launchers
int rexi_grid(int ne, int Bc) {
  const int ct = Bc < 64 ? Bc : 64;
  const int rows_per_pass = (kRWG / 64) * (64 / ct);
  const int tiles = (Bc + 63) / 64;
  int want = (ne + rows_per_pass - 1) / rows_per_pass;
  int cap = 2048 / tiles;
  if (cap < 64) cap = 64;
  int g = want < cap ? want : cap;
  g = (g + 7) / 8 * 8;
  return g > 0 ? g : 8;
}

namespace {
dim3 rgrid(int rows, int Bc) { return dim3(rexi_grid(rows, Bc), (Bc + 63) / 64); }
int flat_grid(size_t n) {
  size_t g = (n + kRWG - 1) / kRWG;
  return (int)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}
// the gather kernels run one row a wave for blocks of 64 or more columns (a
// narrower block would leave lanes idle)
bool uni(int Bc) { return Bc >= 64; }
}  // namespace

void launch_rexi_init(const RexiArgs &a, hipStream_t s) {
  if (uni(a.Bc))
    hipLaunchKernelGGL(k_rexi_init<true>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, a.p);
  else
    hipLaunchKernelGGL(k_rexi_init<false>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, a.p);
}
void launch_rexi_lp(const RexiArgs &a, int kind, hipStream_t s) {
  double2 *y = kind == 0 ? a.r : kind == 1 ? a.v_next : a.t;
  if (uni(a.Bc))
    hipLaunchKernelGGL(k_rexi_lp<true>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, kind, y, a.p);
  else
    hipLaunchKernelGGL(k_rexi_lp<false>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, kind, y, a.p);
}
void launch_rexi_fin_init(const RexiArgs &a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_fin_init, dim3(a.Bc), dim3(kRWG), 0, s, a, nwg);
}
void launch_rexi_v(const RexiArgs &a, hipStream_t s) {
  const dim3 g = rgrid(a.ops.ne, a.Bc);
  hipLaunchKernelGGL(k_rexi_p, g, dim3(kRWG), 0, s, a, a.p, a.v, a.p_next);
  if (uni(a.Bc))
    hipLaunchKernelGGL(k_rexi_sv<true>, g, dim3(kRWG), 0, s, a, a.p_next, a.v_next);
  else
    hipLaunchKernelGGL(k_rexi_sv<false>, g, dim3(kRWG), 0, s, a, a.p_next, a.v_next);
}
void launch_rexi_fin_v(const RexiArgs &a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_fin_v, dim3(a.Bc), dim3(kRWG), 0, s, a, nwg);
}
void launch_rexi_t(const RexiArgs &a, hipStream_t s) {
  if (uni(a.Bc))
    hipLaunchKernelGGL(k_rexi_t<true>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, a.v_next);
  else
    hipLaunchKernelGGL(k_rexi_t<false>, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, a.v_next);
}
void launch_rexi_fin_t(const RexiArgs &a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_fin_t, dim3(a.Bc), dim3(kRWG), 0, s, a, nwg);
}
void launch_rexi_x(const RexiArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_x, rgrid(a.ops.ne, a.Bc), dim3(kRWG), 0, s, a, a.p_next);
}
void launch_rexi_fin_x(const RexiArgs &a, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_fin_x, dim3(a.Bc), dim3(kRWG), 0, s, a, nwg);
}
void launch_rexi_eta(const RexiEtaArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_eta, rgrid(a.ops.nc, a.Bc), dim3(kRWG), 0, s, a);
}
void launch_rexi_combine(const RexiCombineArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_combine, dim3(flat_grid((size_t)a.n * a.ostride)), dim3(kRWG), 0, s, a);
}
void launch_rexi_back(const RexiBackArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_rexi_back, dim3(flat_grid((size_t)a.n * a.Bc)), dim3(kRWG), 0, s, a);
}

}  // namespace pa
