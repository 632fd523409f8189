// HIP kernels of libpa for gfx950 (CDNA4, wave64).
//
// Batched vectors ("blocks") hold Bs columns per row, row-major [row][Bs], so
// a gathered neighbour row is one contiguous run of Bs values: with Bs = 64
// in FP64 a wavefront reads a full 512-byte row per load.  A launch covers a
// column tile of CT = min(Bs, 64) columns (blockIdx.y) and a grid-stride range
// of rows (blockIdx.x); a wave handles RW = 64 / CT rows at a time and lane l
// column l % CT.  Columns carry per-column state (CG scalars, activity), so
// solves of different columns are independent and converged columns freeze.
//
// Per-column sums (CG dot products, residual norms) are deterministic: wave
// shuffles, then LDS across the four waves, then per-workgroup partials with
// plain stores, summed in a fixed order by a later kernel (no floating-point
// atomics).
//
// The single-column Jacobi Chebyshev solves run several steps per launch on
// 512-row parts with rings of halo rows (k_cheb_fused; the row parts and
// rings are built with the operators).
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include <mutex>

#include "pa_kernels.h"

namespace pa {

constexpr int kWG = 256;

struct Lane {
  int ct, rw, col, tile, row0, rstride, rend, lane, wave;
};

// Rows of a launch are split XCD-aware: workgroups are dispatched round-robin
// over the eight XCDs (blockIdx.x % 8), so each XCD gets one contiguous slice
// of rows and each of its workgroups a contiguous block of that slice.  Rows
// that are ELL neighbours (numbered close together) then meet in one XCD's
// L2 instead of being fetched by several.  gridDim.x is a multiple of 8.
__device__ inline Lane lane_map(int Bs, int nrows) {
  Lane L;
  L.ct = Bs < 64 ? Bs : 64;
  L.rw = 64 / L.ct;
  L.lane = threadIdx.x & 63;
  L.wave = threadIdx.x >> 6;
  L.tile = blockIdx.y;
  L.col = L.tile * L.ct + (L.lane % L.ct);
  // Workgroups are dispatched round-robin over the 8 XCDs: XCD k = b & 7
  // owns the contiguous row slice k, and its G/8 workgroups take that slice
  // in interleaved passes (workgroup w: passes w, w + G/8, ...), so the rows
  // an XCD works on at any moment form one window and the neighbour gathers
  // stay in its L2.
  const int G = gridDim.x, per = G >> 3;
  const int xcd = blockIdx.x & 7, w = blockIdx.x >> 3;
  const int slice = (nrows + 7) >> 3;
  const int rpp = (kWG / 64) * L.rw;  // rows of one workgroup pass
  const int rbeg = xcd * slice + w * rpp;
  L.rend = min(nrows, (xcd + 1) * slice);
  L.row0 = rbeg + L.wave * L.rw + L.lane / L.ct;
  L.rstride = per * rpp;
  return L;
}

// A read-only table seen through the constant address space: loads at
// wave-uniform addresses then go through the scalar unit into scalar
// registers (as vector loads every lane would receive its own copy of the
// value, through the vector memory path).
template <typename T>
__device__ inline const __attribute__((address_space(4))) T *uniform_ro(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

// Row tables of the block kernels.  UNI: at least 64 columns (lane_map gives
// a wave one row), so the row number is made wave-uniform and the row's
// operator entries load through the scalar unit.
template <bool UNI>
__device__ inline int urow(int e) {
  return UNI ? __builtin_amdgcn_readfirstlane(e) : e;
}
template <bool UNI, typename T>
__device__ inline T rl(const T *p, size_t i) {
  if constexpr (UNI)
    return uniform_ro(p)[i];
  else
    return p[i];
}

template <bool UNI>
__device__ inline uint2 rl(const uint2 *p, size_t i) {
  if constexpr (UNI) {
    const unsigned long long v = uniform_ro(reinterpret_cast<const unsigned long long *>(p))[i];
    return make_uint2((unsigned)v, (unsigned)(v >> 32));
  } else {
    return p[i];
  }
}

// Sum v over lanes that share a column (lane % ct), result valid in lanes < ct.
__device__ inline double wave_col_sum(double v, int ct) {
  for (int off = 32; off >= ct; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum v over aligned groups of G lanes (G a power of two <= 64); the result
// is valid in the first lane of each group.
__device__ inline double lane_group_sum(double v, int G) {
  for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

// Per-workgroup column sums of NQ quantities: wave shuffles, then LDS over the
// four waves, stored to part[tile][wg][q][64] with plain stores.  The
// cross-workgroup sum is done by k_finalize after the kernel boundary, which
// gives the coherence that per-workgroup device-scope fences would otherwise
// buy with an L2 write-back and invalidate per workgroup.
template <int NQ>
__device__ void wg_partials(const Lane &L, double (&v)[NQ], double *part, int max_wg) {
  __shared__ double red[NQ][kWG / 64][64];
  for (int q = 0; q < NQ; q++) {
    double s = wave_col_sum(v[q], L.ct);
    if (L.lane < L.ct) red[q][L.wave][L.lane] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NQ * 64; idx += kWG) {
    const int q = idx / 64, c = idx % 64;
    if (c < L.ct) {
      double s = 0;
      for (int w = 0; w < kWG / 64; w++) s += red[q][w][c];
      part[(((size_t)L.tile * max_wg + blockIdx.x) * NQ + q) * 64 + c] = s;
    }
  }
}

// Measurement hook: the first workgroup of each tile adds the tile's active
// columns to prof[0]; tile 0 counts the launch in prof[1].
__device__ void count_active(const Lane &L, SolveState st) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned n = 0;
    for (int j = 0; j < L.ct; j++) n += st.active[L.tile * L.ct + j] ? 1u : 0u;
    atomicAdd(&st.prof[0], n);
    if (L.tile == 0) atomicAdd(&st.prof[1], 1u);
  }
}

// Per column: |r_final|^2 <= rtol^2 |r_0|^2, else count a failure.
__device__ void check_block(const CheckArgs &a, int blk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ct = a.Bs < 64 ? a.Bs : 64;
  const int cpb = ct < 4 ? ct : 4;
  const int bpt = ct / cpb;
  const int tile = blk / bpt;
  // the waves of a block share its cpb columns: column cl = base + (wave % cpb),
  // and the 4 / cpb waves of one column split the workgroup partials
  const int split = 4 / cpb;
  const int cl = (blk % bpt) * cpb + wave % cpb;
  const int part = wave / cpb;
  const int c = tile * ct + cl;
  double b = 0.0, r = 0.0;
  // the first four waves do the check (workgroups of more waves call it too)
  const bool on = wave < 4;
  for (int w = part * 64 + lane; on && w < a.nwg_init; w += 64 * split)
    b += a.part_init[((size_t)tile * a.max_wg + w) * 64 + cl];
  for (int w = part * 64 + lane; on && w < a.nwg_last; w += 64 * split)
    r += a.part_last[((size_t)tile * a.max_wg + w) * 64 + cl];
  b = wave_col_sum(b, 1);
  r = wave_col_sum(r, 1);
  __shared__ double red[2][4];
  if (on && lane == 0) {
    red[0][wave] = b;
    red[1][wave] = r;
  }
  __syncthreads();
  if (on && part == 0 && lane == 0) {
    b = 0.0;
    r = 0.0;
    for (int p = 0; p < split; p++) {  // fixed order
      b += red[0][p * cpb + wave];
      r += red[1][p * cpb + wave];
    }
    if (a.colK[c] >= a.kneed && b > 0.0) {
      const double rel = sqrt(r / b);
      a.resid[c] = rel;
      // non-negative doubles order like their bit patterns
      if (a.resid_max) atomicMax(a.resid_max, (unsigned long long)__double_as_longlong(rel));
      if (!(r <= a.rtol2 * b)) atomicAdd(a.fail, 1);
    }
  }
}

__global__ __launch_bounds__(kWG) void k_cheb_check(CheckArgs a) { check_block(a, blockIdx.x); }

// The previous solve's check, folded into a set-up kernel: its first
// chk_blocks workgroups (over the whole grid) each do one check block.
__device__ inline void folded_check(const CheckArgs &a, int blocks) {
  if (blocks <= 0) return;
  const int bi = blockIdx.y * gridDim.x + blockIdx.x;
  if (bi < blocks) check_block(a, bi);
}

// ---------------------------------------------------------------- stiffness
// The stiffness arithmetic of one row, in one fixed rounding order for every
// kernel that forms it (no contraction left to the compiler).
#pragma clang fp contract(off)
// velocity row: scale (-sum_j F_j u_j + g (eta_0 - eta_1)); fu = sum_j F_j u_j
// accumulated by fma in ELL order
__device__ inline double stiff_u(double scale, double fu, double g, double eta0, double eta1) {
  return scale * fma(g, eta0 - eta1, -fu);
}
// depth row: scale (-H div / |c|) + addA + addB (an absent addend is 0)
__device__ inline double stiff_eta(double scale, double H, double div, double inv_area, double addA,
                                   double addB) {
  return (scale * ((-H * div) * inv_area) + addA) + addB;
}
// d_0 = theta_inv D^-1 r_0
__device__ inline double stiff_d0(double theta_inv, double dinv, double r) { return (theta_inv * dinv) * r; }
#pragma clang fp contract(on)


// One application of the linear operator with the mass solve set up:
//   velocity: r = scale (-F u + g D' eta), out_u = addA_u + addB_u (CG start),
//   depth:    out_eta = scale (-H D u / |c|) + addA_eta + addB_eta,
// for columns with colK[c] >= kneed; optionally acc += coef * in (grouped
// column sums of G columns) for columns with colK[c] >= acc_k.
template <bool UNI>
__global__ __launch_bounds__(kWG) void k_stiff(StiffArgs a) {
  folded_check(a.chk, a.chk_blocks);
  const Lane L = lane_map(a.Bs, a.ops.ne > a.ops.nc ? a.ops.ne : a.ops.nc);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  const bool act = a.colK[c] >= a.kneed;
  const bool acc_on = a.acc_u != nullptr && a.colK[c] >= a.acc_k;
  const double coef = acc_on ? a.coef[c] : 0.0;
  double rr = 0.0;
  for (int base = L.row0 - L.lane / L.ct; base < L.rend; base += L.rstride) {
    const int e = urow<UNI>(base + L.lane / L.ct);
    // edges
    double accv = 0.0;
    if (e < o.ne && e < L.rend) {
      const size_t ie = (size_t)e * Bs + c;
      if (act) {
        double fu = 0.0;
#pragma unroll
        for (int j = 0; j < 5; j++)
          fu = fma(rl<UNI>(o.cor, 5 * e + j), a.in_u[(size_t)rl<UNI>(o.ell_col, 5 * e + j) * Bs + c], fu);
        const int c0 = rl<UNI>(o.ecell, 2 * e), c1 = rl<UNI>(o.ecell, 2 * e + 1);
        const double r = stiff_u(a.scale, fu, o.g, a.in_eta[(size_t)c0 * Bs + c], a.in_eta[(size_t)c1 * Bs + c]);
        double x0 = 0.0;
        if (a.addA_u) x0 += a.addA_u[ie];
        if (a.addB_u) x0 += a.addB_u[ie];
        a.r[ie] = r;
        a.out_u[ie] = x0;
        if (a.d0) {
          a.d0[ie] = stiff_d0(a.theta_inv, rl<UNI>(o.dinv, e), r);
          rr = fma(r, r, rr);
        }
      }
      if (acc_on) accv = coef * a.in_u[ie];
    }
    if (a.acc_u) {
      double s = lane_group_sum(accv, a.G);
      if (e < o.ne && e < L.rend && (c % a.G) == 0)
        a.acc_u[(size_t)e * (Bs / a.G) + c / a.G] += s;
    }
    // cells
    double acce = 0.0;
    if (e < o.nc && e < L.rend) {
      const int t = e;
      const size_t it = (size_t)t * Bs + c;
      if (act) {
        double div = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++)
          div = fma((double)rl<UNI>(o.csgn, 3 * t + j), a.in_u[(size_t)rl<UNI>(o.cedge, 3 * t + j) * Bs + c], div);
        a.out_eta[it] = stiff_eta(a.scale, o.H, div, rl<UNI>(o.inv_area, t), a.addA_eta ? a.addA_eta[it] : 0.0,
                                  a.addB_eta ? a.addB_eta[it] : 0.0);
      }
      if (acc_on) acce = coef * a.in_eta[it];
    }
    if (a.acc_u) {
      double s = lane_group_sum(acce, a.G);
      if (e < o.nc && e < L.rend && (c % a.G) == 0)
        a.acc_eta[(size_t)e * (Bs / a.G) + c / a.G] += s;
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.st.cnt[1] = 0;
  if (a.part_rr) {
    double v[1] = {rr};
    wg_partials<1>(L, v, a.part_rr, a.max_wg);
  }
}

// -------------------------------------------- Chebyshev semi-iteration
// Reduction-free solver for the velocity mass matrix M: with spectral bounds
// [lmin, lmax] of D^-1 M (theta, delta their centre and half-width,
// sigma = theta/delta), from r_0 and d_0 = D^-1 r_0 / theta,
//   x += d_k,  r -= M d_k,  d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^-1 r,
//   rho_0 = 1/sigma,  rho_{k+1} = 1/(2 sigma - rho_k)
// (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1).  The step
// count follows from the bounds; the final residual is checked in FP64.  One
// kernel per step, gathering only d.
// Direction update of the Jacobi Chebyshev step.
__device__ inline double cheb_dir(double c1, double c2, double d, double dinv, double r) {
  // one fixed rounding order at every call site (no contraction left to the
  // compiler), so that a row's direction is the same bits in every kernel
  return fma(c1, d, (c2 * dinv) * r);
}

__global__ __launch_bounds__(kWG) void k_cheb_iter(ChebArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  if (a.prof && blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned n = 0;
    for (int j = 0; j < L.ct; j++) n += a.colK[L.tile * L.ct + j] >= a.kneed ? 1u : 0u;
    atomicAdd(&a.prof[a.last ? 2 : 0], n);
    if (L.tile == 0) atomicAdd(&a.prof[1], 1u);
  }
  double sums[1] = {0.0};
  if (a.colK[c] >= a.kneed) {
    for (int e = L.row0; e < L.rend; e += L.rstride) {
      double q = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) q = fma(o.mass[5 * e + j], a.d_in[(size_t)o.ell_col[5 * e + j] * Bs + c], q);
      const size_t ie = (size_t)e * Bs + c;
      const double d = a.d_in[ie];
      a.x[ie] += d;
      const double r = a.r[ie] - q;
      a.r[ie] = r;
      if (a.last)
        sums[0] += r * r;
      else if (!a.nodir)
        a.d_out[ie] = cheb_dir(a.c1, a.c2, d, o.dinv[e], r);
    }
  }
  if (a.last) wg_partials<1>(L, sums, a.part, a.max_wg);
}

// S steps of the single-column Jacobi semi-iteration in one launch.  A step
// costs little beyond its launch and the latency of its dependent gather, so
// fusing steps divides both.  Workgroup p owns the kPartRows rows of part p.
// Step 1 runs on the part and its rings 1..S-1 from the previous launch's r
// and d (gathered from global memory):
//   r' = r - M d,  d' = c1 d + c2 D^-1 r',
// step s > 1 on the part and rings 1..S-s, gathering the previous step's d
// from LDS; x += d of each step on the part's rows.  A ring row's values are
// formed again by the workgroup that owns that row, in the same order, hence
// bit for bit the same as one step per launch.  Ring rows read r and d of the
// previous launch, which no workgroup writes in this one: the part's new r
// and d go to separate output buffers.  Parts are laid over the XCDs like
// lane_map's slices (XCD k takes parts k per .. k per + per - 1), so
// neighbouring parts and their rings share an L2.
constexpr int kFWG = kPartRows;  // workgroup size of the fused kernel: one row a thread
constexpr int kRingSlots = kHaloMax / kFWG;  // ring rows per thread

// NSLOT: ring slots of kFWG rows the launch's first step covers (every part's
// rings 1..S-1 fit).  The loads go out in three waves by dependence (indices
// and row values; the ring rows they name and the own row's gathers; the
// ring rows' gathers); a ring slot past the part's rings (list entry -1)
// loads nothing, and a wave skips a slot in a later step when all its rows
// lie past the rings that take that step.  Ring rows that no later step
// reads work anyway (nothing reads their results), and the stores to global
// memory are predicated (an inactive column; the threads past a ragged last
// part, which work on a copy of its last row).
template <int NSLOT, bool SETUP>
__global__ __launch_bounds__(kFWG) void k_cheb_fused(ChebFusedArgs a) {
  const DevOps &o = a.ops;
  const int t = threadIdx.x;
  if (a.prof && blockIdx.x == 0 && t == 0) {
    const bool on = a.colK[0] >= a.kneed;
    atomicAdd(&a.prof[a.last ? 2 : 0], on ? 1u : 0u);
    atomicAdd(&a.prof[1], 1u);
    if (on) atomicAdd(a.prof_bytes, a.bytes);
  }
  const bool act = a.colK[0] >= a.kneed;
  const int per = gridDim.x >> 3;
  const int p = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const int S = a.S;
  __shared__ double dl[2][kPartRows + kHaloMax];
  __shared__ double red[2][kFWG / 64];
  double s2 = 0.0, s0 = 0.0;
  // the previous solve's residual check runs in the workgroups past the last
  // part (the grid of a set-up launch has chk_blocks of them), beside the
  // parts' work instead of before one part's
  if (SETUP && p >= o.hparts && p - o.hparts < a.chk_blocks) check_block(a.chk, p - o.hparts);
  if (p < o.hparts) {
    const int e0 = p * kPartRows;
    const bool own = e0 + t < o.ne;
    const int e = own ? e0 + t : o.ne - 1;
    const int32_t *rrow = o.ring_row + (size_t)p * kHaloMax;
    const uint16_t *rloc = o.ring_loc + (size_t)p * kHaloMax * 5;
    // ring counts of the part (rows of rings 1..r), first needed at step 2
    int cnt[kFusedMax - 1];
#pragma unroll
    for (int i = 0; i < kFusedMax - 1; i++) cnt[i] = o.ring_cnt[8 * p + i];
    const int wrow = __builtin_amdgcn_readfirstlane(t & ~63);  // the wave's first row in a slot
    constexpr int NS = NSLOT > 0 ? NSLOT : 1;
    // first wave of loads: the own row (ELL slot 0 is the row itself) and
    // the ring rows' numbers; with SETUP also the Coriolis row, the row's
    // cells and the addends of x_0, and the part's depth row
    double m[5], fc[5];
    int col[5], lc[5], ec[2];
#pragma unroll
    for (int j = 0; j < 5; j++) {
      col[j] = o.ell_col[5 * e + j];
      m[j] = o.mass[5 * e + j];
      lc[j] = o.hloc[(size_t)j * o.ne + e];
      if (SETUP) fc[j] = o.cor[5 * e + j];
    }
    const double dinv = o.dinv[e];
    double dv = 0.0, x, r;
    if (SETUP) {
      ec[0] = o.ecell[2 * e];
      ec[1] = o.ecell[2 * e + 1];
      x = 0.0;
      if (a.addA_u) x += a.addA_u[e];
      if (a.addB_u) x += a.addB_u[e];
    } else {
      dv = a.d_in[e];
      x = a.x[e];
      r = a.r_in[e];
    }
    const int cell = p * a.cpp + t;
    const bool cown = SETUP && t < a.cpp && cell < o.nc;
    const int cc = cown ? cell : 0;
    int cedge[3];
    double csg[3], cia = 0.0;
    if (SETUP) {
#pragma unroll
      for (int j = 0; j < 3; j++) {
        cedge[j] = o.cedge[3 * cc + j];
        csg[j] = (double)o.csgn[3 * cc + j];
      }
      cia = o.inv_area[cc];
    }
    int g[NS];
#pragma unroll
    for (int q = 0; q < NSLOT; q++) g[q] = rrow[t + q * kFWG];
    // second wave: the ring rows, the own row's gathers
    double rm[NS][5], rdinv[NS], rr[NS], dg[NS], rfc[NS][5];
    int gc[NS][5], rlc[NS][5], rec[NS][2];
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
      const int h = t + q * kFWG;
      dg[q] = rdinv[q] = rr[q] = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) {
        gc[q][j] = rlc[q][j] = 0;
        rm[q][j] = rfc[q][j] = 0.0;
      }
      rec[q][0] = rec[q][1] = 0;
      if (g[q] >= 0) {  // past the part's rings the list holds -1
#pragma unroll
        for (int j = 0; j < 5; j++) {
          gc[q][j] = o.ell_col[5 * g[q] + j];
          if (!SETUP) rm[q][j] = o.mass[5 * g[q] + j];
          rlc[q][j] = rloc[5 * h + j];
          if (SETUP) rfc[q][j] = o.cor[5 * g[q] + j];
        }
        rdinv[q] = o.dinv[g[q]];
        if (SETUP) {
          rec[q][0] = o.ecell[2 * g[q]];
          rec[q][1] = o.ecell[2 * g[q] + 1];
        } else {
          dg[q] = a.d_in[g[q]];
          rr[q] = a.r_in[g[q]];
        }
      }
    }
    if (SETUP) {
      // step 1 = the set-up: r_0, d_0 (own row), and the part's depth rows
      double fu = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) fu = fma(fc[j], a.in_u[col[j]], fu);
      r = stiff_u(a.scale, fu, o.g, a.in_eta[ec[0]], a.in_eta[ec[1]]);
      s0 = fma(r, r, s0);
      dl[0][t] = stiff_d0(a.theta_inv, dinv, r);
      double div = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) div = fma(csg[j], a.in_u[cedge[j]], div);
      if (cown && act)
        a.out_eta[cc] = stiff_eta(a.scale, o.H, div, cia, a.addA_eta ? a.addA_eta[cc] : 0.0,
                                  a.addB_eta ? a.addB_eta[cc] : 0.0);
    } else {
      double q0 = fma(m[0], dv, 0.0);
#pragma unroll
      for (int j = 1; j < 5; j++) q0 = fma(m[j], a.d_in[col[j]], q0);
      x += dv;
      r -= q0;
      if (S > 1) dl[0][t] = cheb_dir(a.c1[0], a.c2[0], dv, dinv, r);
    }
    // third wave: the ring rows' gathers; step 1 on rings 1..S-1 (ring row
    // h = t + q kFWG stays in slot q of thread t, its matrix row, local
    // columns, diagonal and residual in registers, so that later steps touch
    // only LDS)
#pragma unroll
    for (int q = 0; q < NSLOT; q++)
      if (g[q] >= 0) {
        double dn1;
        if (SETUP) {
          double fu = 0.0;
#pragma unroll
          for (int j = 0; j < 5; j++) fu = fma(rfc[q][j], a.in_u[gc[q][j]], fu);
          rr[q] = stiff_u(a.scale, fu, o.g, a.in_eta[rec[q][0]], a.in_eta[rec[q][1]]);
          dn1 = stiff_d0(a.theta_inv, rdinv[q], rr[q]);
        } else {
          double qs = fma(rm[q][0], dg[q], 0.0);
#pragma unroll
          for (int j = 1; j < 5; j++) qs = fma(rm[q][j], a.d_in[gc[q][j]], qs);
          rr[q] -= qs;
          dn1 = cheb_dir(a.c1[0], a.c2[0], dg[q], rdinv[q], rr[q]);
        }
        dl[0][kPartRows + t + q * kFWG] = dn1;
      }
    // with SETUP the ring rows' mass rows load only now, after the Coriolis
    // rows are done with (fewer registers live at once)
    if (SETUP) {
#pragma unroll
      for (int q = 0; q < NSLOT; q++)
        if (g[q] >= 0) {
#pragma unroll
          for (int j = 0; j < 5; j++) rm[q][j] = o.mass[5 * g[q] + j];
        }
    }
    for (int st = 1; st < S; st++) {
      __syncthreads();
      const double *dp = dl[(st - 1) & 1];
      double *dn = dl[st & 1];
      const double c1 = a.c1[st], c2 = a.c2[st];
      // every LDS read of the step before its first write (the compiler
      // cannot tell the two halves of dl apart); a wave skips the slots whose
      // 64 rows all lie past the rings that take this step
      const int nh = st + 1 < S ? cnt[S - 2 - st] : 0;
      double dq[5], dr[NS][5];
#pragma unroll
      for (int j = 0; j < 5; j++) dq[j] = dp[j ? lc[j] : t];
#pragma unroll
      for (int k = 0; k < NSLOT; k++)
        if (k * kFWG + wrow < nh) {
#pragma unroll
          for (int j = 0; j < 5; j++) dr[k][j] = dp[j ? rlc[k][j] : kPartRows + t + k * kFWG];
        }
      dv = dq[0];
      double q = fma(m[0], dv, 0.0);
#pragma unroll
      for (int j = 1; j < 5; j++) q = fma(m[j], dq[j], q);
      x += dv;
      r -= q;
      // rings 1..S-1-st take this step too (rows past them are not read)
      double dnr[NS];
#pragma unroll
      for (int k = 0; k < NSLOT; k++)
        if (k * kFWG + wrow < nh) {
          double qs = fma(rm[k][0], dr[k][0], 0.0);
#pragma unroll
          for (int j = 1; j < 5; j++) qs = fma(rm[k][j], dr[k][j], qs);
          rr[k] -= qs;
          dnr[k] = cheb_dir(c1, c2, dr[k][0], rdinv[k], rr[k]);
        }
      if (st + 1 < S) dn[t] = cheb_dir(c1, c2, dv, dinv, r);
#pragma unroll
      for (int k = 0; k < NSLOT; k++)
        if (k * kFWG + wrow < nh) dn[kPartRows + t + k * kFWG] = dnr[k];
    }
    if (own && act) {
      a.x[e] = x;
      a.r_out[e] = r;
      if (a.last)
        s2 = r * r;
      else
        a.d_out[e] = cheb_dir(a.c1[S - 1], a.c2[S - 1], dv, dinv, r);
    }
    if (!own) s0 = 0.0;
  }
  if (a.last || SETUP) {
    // partials of r.r (and with SETUP of r_0.r_0) per workgroup, at the
    // place of tile 0, column 0 of wg_partials' layout
    s2 = wave_col_sum(s2, 1);
    s0 = wave_col_sum(s0, 1);
    if ((t & 63) == 0) {
      red[0][t >> 6] = s2;
      red[1][t >> 6] = s0;
    }
    __syncthreads();
    if (t == 0) {
      double w = 0.0, w0 = 0.0;
      for (int i = 0; i < kFWG / 64; i++) {
        w += red[0][i];
        w0 += red[1][i];
      }
      if (a.last) a.part[(size_t)blockIdx.x * 64] = w;
      if (SETUP) a.part_rr[(size_t)blockIdx.x * 64] = w0;
    }
  }
}

// The Jacobi semi-iteration of a block in three-term form.  With y the
// increment of x over x_0 (y_1 = d_0 from the set-up kernel) and
// d_i = y_{i+1} - y_i, the two-term step (x += d, r -= M d,
// d' = c1 d + c2 D^-1 r) becomes
//   y_{i+1} = y_i + c1 (y_i - y_{i-1}) + c2 D^-1 (b - M y_i),  b = r_0,
// which reads y_i, y_{i-1} and b and writes y_{i+1} (four vectors a step
// against six); the residual b - M y_i is formed in registers.  The
// finishing launch adds x += y_K and sums the true final residual.
template <bool UNI>
__global__ __launch_bounds__(kWG) void k_cheb3_iter(Cheb3Args a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  if (a.prof && blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned n = 0;
    for (int j = 0; j < L.ct; j++) n += a.colK[L.tile * L.ct + j] >= a.kneed ? 1u : 0u;
    atomicAdd(&a.prof[a.finish ? 2 : 0], n);
    if (L.tile == 0) atomicAdd(&a.prof[1], 1u);
    // per active column and row: y (and y_prev unless zero), b, y' or x in
    // and out; per row and tile: the ELL row and (steps) the diagonal
    const unsigned long long pc = a.finish ? 32 : (a.zero_prev ? 24 : 32);
    atomicAdd(a.prof_bytes, (unsigned long long)o.ne * (pc * n + (a.finish ? 60 : 68)));
  }
  double sums[1] = {0.0};
  if (a.colK[c] >= a.kneed) {
    for (int el = L.row0; el < L.rend; el += L.rstride) {
      const int e = urow<UNI>(el);
      const size_t ie = (size_t)e * Bs + c;
      const double yc = a.y_cur[ie];
      double q = fma(rl<UNI>(o.mass, 5 * e), yc, 0.0);
#pragma unroll
      for (int j = 1; j < 5; j++)
        q = fma(rl<UNI>(o.mass, 5 * e + j), a.y_cur[(size_t)rl<UNI>(o.ell_col, 5 * e + j) * Bs + c], q);
      const double r = a.b[ie] - q;
      if (a.finish) {
        a.x[ie] += yc;
        sums[0] = fma(r, r, sums[0]);
      } else {
        const double yp = a.zero_prev ? 0.0 : a.y_prev[ie];
        a.y_next[ie] = fma(a.c1, yc - yp, yc) + (a.c2 * rl<UNI>(o.dinv, e)) * r;
      }
    }
  }
  if (a.finish) wg_partials<1>(L, sums, a.part, a.max_wg);
}

// The same semi-iteration preconditioned by the learned P = G G^T:
//   x += d_k,  r_{k+1} = r_k - M d_k,  d_{k+1} = c1 d_k + c2 P r_{k+1},
// with P r_{k+1} formed as P r_k - (P M) d_k so that one kernel per step
// suffices (both products gather only values of the previous step; P and
// P M are stored explicitly, column-major ELL, FP32 values).  M d_k and the
// residual update stay FP64 with the FP64 matrix, so r is a true FP64
// residual; the FP32 rounding of P and P M only perturbs the preconditioner.
// sum_j val_j v[col_j] over W packed entries of row e (column-major table);
// W > 0: fixed width, every load issued before the first use.
template <int W, bool UNI>
__device__ inline double lp_row_dot(const uint2 *t, int w, int ne, int e, const double *v, int Bs, int c) {
  double z = 0.0;
  if constexpr (W > 0) {
    uint2 q[W];
#pragma unroll
    for (int j = 0; j < W; j++) q[j] = rl<UNI>(t, (size_t)j * ne + e);
#pragma unroll
    for (int j = 0; j < W; j++) z += (double)__uint_as_float(q[j].y) * v[(size_t)q[j].x * Bs + c];
  } else {
    for (int j = 0; j < w; j++) {
      const uint2 q = rl<UNI>(t, (size_t)j * ne + e);
      z += (double)__uint_as_float(q.y) * v[(size_t)q.x * Bs + c];
    }
  }
  return z;
}

template <int WP, int WPM, bool UNI>
__global__ __launch_bounds__(kWG) void k_cheb_lp_iter(ChebLpArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs, ne = o.ne;
  if (a.prof && blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned n = 0;
    for (int j = 0; j < L.ct; j++) n += a.colK[L.tile * L.ct + j] >= a.kneed ? 1u : 0u;
    atomicAdd(&a.prof[a.last ? 2 : 0], n);
    if (L.tile == 0) atomicAdd(&a.prof[1], 1u);
  }
  const double *__restrict__ rin = a.r_in;
  const double *__restrict__ din = a.d_in;
  const uint2 *__restrict__ tp = a.lp.p;
  const uint2 *__restrict__ tpm = a.lp.pm;
  double sums[1] = {0.0};
  if (a.colK[c] >= a.kneed) {
    for (int el = L.row0; el < L.rend; el += L.rstride) {
      const int e = urow<UNI>(el);
      // every table entry and gathered operand is loaded before any store
      int mc[5];
      double mv[5], dg[5];
#pragma unroll
      for (int j = 0; j < 5; j++) {
        mc[j] = rl<UNI>(o.ell_col, 5 * e + j);
        mv[j] = rl<UNI>(o.mass, 5 * e + j);
      }
      const size_t ie = (size_t)e * Bs + c;
      const double d = din[ie], r0 = rin[ie], x0 = a.x[ie];
#pragma unroll
      for (int j = 0; j < 5; j++) dg[j] = din[(size_t)mc[j] * Bs + c];
      double z = 0.0;
      if (!a.last) {
        if constexpr (WP > 0 && WPM > 0) {
          uint2 qp[WP], qm[WPM];
#pragma unroll
          for (int j = 0; j < WP; j++) qp[j] = rl<UNI>(tp, (size_t)j * ne + e);
#pragma unroll
          for (int j = 0; j < WPM; j++) qm[j] = rl<UNI>(tpm, (size_t)j * ne + e);
          double gp[WP], gm[WPM];
#pragma unroll
          for (int j = 0; j < WP; j++) gp[j] = rin[(size_t)qp[j].x * Bs + c];
#pragma unroll
          for (int j = 0; j < WPM; j++) gm[j] = din[(size_t)qm[j].x * Bs + c];
#pragma unroll
          for (int j = 0; j < WP; j++) z += (double)__uint_as_float(qp[j].y) * gp[j];
#pragma unroll
          for (int j = 0; j < WPM; j++) z -= (double)__uint_as_float(qm[j].y) * gm[j];
        } else {
          z = lp_row_dot<0, UNI>(tp, a.lp.wp, ne, e, rin, Bs, c) - lp_row_dot<0, UNI>(tpm, a.lp.wpm, ne, e, din, Bs, c);
        }
      }
      double q = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) q += mv[j] * dg[j];
      const double r = r0 - q;
      a.x[ie] = x0 + d;
      a.r_out[ie] = r;
      if (a.last)
        sums[0] += r * r;
      else
        a.d_out[ie] = a.c1 * d + a.c2 * z;
    }
  }
  if (a.last) wg_partials<1>(L, sums, a.part, a.max_wg);
}

template <int WP, bool UNI>
__global__ __launch_bounds__(kWG) void k_lp_dir(LpDirArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const int c = L.col, Bs = a.Bs, ne = a.ops.ne;
  if (a.colK[c] < a.kneed) return;
  for (int el = L.row0; el < L.rend; el += L.rstride) {
    const int e = urow<UNI>(el);
    const size_t ie = (size_t)e * Bs + c;
    const double z = lp_row_dot<WP, UNI>(a.lp.p, a.lp.wp, ne, e, a.r, Bs, c);
    a.d_out[ie] = (a.c1 != 0.0 ? a.c1 * a.d_in[ie] : 0.0) + a.c2 * z;
  }
}


// ----------------------------------- FP32 inner solves, FP64 refinement
// Mixed-precision mass solve: the correction equation M d = r is solved
// approximately by the Chebyshev semi-iteration in FP32 (FP32 copy of M,
// FP32 vectors), the correction is added to x in FP64 and the residual
// updated with the FP64 matrix, r -= M x32, so the outer residual is a true
// FP64 residual; a final check compares it with the tolerance.
// The inner FP32 solve in the three-term form of the same semi-iteration:
// with d_i = x_{i+1} - x_i the step x += d_i, r -= M d_i,
// d_{i+1} = c1 d_i + c2 D^-1 r becomes
//   x_{i+1} = x_i + c1 (x_i - x_{i-1}) + c2 D^-1 (b - M x_i),
// which reads x_i, x_{i-1} and b and writes x_{i+1} (a quarter of the bytes
// of the two-term step that keeps x, r and d; the residual is formed in
// registers).  x_1 = D^-1 b / theta comes from the refinement kernel.
// Measurement hook of the FP32 steps: per active column and row x_i,
// x_{i-1} (unless zero), b and x_{i+1} in FP32; per row the FP32 ELL row
// (5 columns, 5 values) and diagonal.
__device__ inline void cheb32_prof(const Cheb32Args &a, int ncols_active) {
  atomicAdd(&a.prof[0], (unsigned)ncols_active);
  atomicAdd(&a.prof[1], 1u);
  const unsigned long long pc = a.zero_prev ? 12 : 16;
  atomicAdd(a.prof_bytes, (unsigned long long)a.ops.ne * (pc * ncols_active + 44));
}

__global__ __launch_bounds__(kWG) void k_cheb32_iter(Cheb32Args a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  if (a.prof && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    int n = 0;
    for (int j = 0; j < Bs; j++) n += a.colK[j] >= a.kneed ? 1 : 0;
    cheb32_prof(a, n);
  }
  if (a.colK[c] < a.kneed) return;
  for (int e = L.row0; e < L.rend; e += L.rstride) {
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < 5; j++) q += o.mass32[5 * e + j] * a.x_cur[(size_t)o.ell_col[5 * e + j] * Bs + c];
    const size_t ie = (size_t)e * Bs + c;
    const float xc = a.x_cur[ie];
    const float xp = a.zero_prev ? 0.0f : a.x_prev[ie];
    a.x_next[ie] = xc + a.c1 * (xc - xp) + a.c2 * o.dinv32[e] * (a.b32[ie] - q);
  }
}

// The same step on four adjacent columns per lane (blocks of at least eight
// columns): a row of Bs FP32 values is Bs/4 float4s, so the row mapping of a
// block of Bs/4 columns applies and every load and store moves 16 bytes.
// A group with any active column is computed whole: the FP32 scratch of
// inactive columns is never read back (the refinement and the final check
// skip them).
__device__ inline float4 f4_fma(float m, float4 v, float4 q) {
  q.x += m * v.x;
  q.y += m * v.y;
  q.z += m * v.z;
  q.w += m * v.w;
  return q;
}

template <bool UNI>
__global__ __launch_bounds__(kWG) void k_cheb32_iter4(Cheb32Args a) {
  const int Bq = a.Bs >> 2;
  const Lane L = lane_map(Bq, a.ops.ne);
  const DevOps &o = a.ops;
  const int cq = L.col, c0 = 4 * cq;
  if (a.prof && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    int n = 0;
    for (int j = 0; j < a.Bs; j++) n += a.colK[j] >= a.kneed ? 1 : 0;
    cheb32_prof(a, n);
  }
  if (a.colK[c0] < a.kneed && a.colK[c0 + 1] < a.kneed && a.colK[c0 + 2] < a.kneed &&
      a.colK[c0 + 3] < a.kneed)
    return;
  const float4 *__restrict__ xcur = (const float4 *)a.x_cur;
  const float4 *xprev = (const float4 *)a.x_prev;
  const float4 *b4 = (const float4 *)a.b32;
  float4 *xnext = (float4 *)a.x_next;
  for (int el = L.row0; el < L.rend; el += L.rstride) {
    const int e = urow<UNI>(el);
    float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int j = 0; j < 5; j++)
      q = f4_fma(rl<UNI>(o.mass32, 5 * e + j), xcur[(size_t)rl<UNI>(o.ell_col, 5 * e + j) * Bq + cq], q);
    const size_t ie = (size_t)e * Bq + cq;
    const float4 xc = xcur[ie];
    const float4 xp = a.zero_prev ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : xprev[ie];
    const float4 bv = b4[ie];
    const float g = a.c2 * rl<UNI>(o.dinv32, e);
    xnext[ie] = make_float4(xc.x + a.c1 * (xc.x - xp.x) + g * (bv.x - q.x),
                            xc.y + a.c1 * (xc.y - xp.y) + g * (bv.y - q.y),
                            xc.z + a.c1 * (xc.z - xp.z) + g * (bv.z - q.z),
                            xc.w + a.c1 * (xc.w - xp.w) + g * (bv.w - q.w));
  }
}

template <bool UNI>
__global__ __launch_bounds__(kWG) void k_refine(RefineArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  double sums[1] = {0.0};
  if (a.colK[c] >= a.kneed) {
    for (int el = L.row0; el < L.rend; el += L.rstride) {
      const int e = urow<UNI>(el);
      const size_t ie = (size_t)e * Bs + c;
      double r = a.r[ie];
      if (!a.first) {
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < 5; j++)
          q += rl<UNI>(o.mass, 5 * e + j) * (double)a.x32[(size_t)rl<UNI>(o.ell_col, 5 * e + j) * Bs + c];
        a.x[ie] = a.x_zero ? (double)a.x32[ie] : a.x[ie] + (double)a.x32[ie];
        r -= q;
        if (!a.last) a.r[ie] = r;  // the last residual only feeds the check
      }
      if (a.last) {
        sums[0] += r * r;
      } else {
        const float r32 = (float)r;
        a.r32[ie] = r32;
        a.d32[ie] = a.theta_inv * rl<UNI>(o.dinv32, e) * r32;
      }
    }
  }
  if (a.last) wg_partials<1>(L, sums, a.part, a.max_wg);
}

// -------------------------------------------------- CG (Chronopoulos-Gear)
// Jacobi-preconditioned CG in the single-reduction form of Chronopoulos and
// Gear: with u = D^-1 r and w = M u,
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u' = D^-1 r,  w' = M u',  gamma' = r'.u',  delta' = w'.u',
//   beta' = gamma'/gamma,  alpha' = gamma' / (delta' - beta' gamma'/alpha).
// One kernel per iteration.  u' at the five ELL neighbours is recomputed from
// the previous iteration's r, w and s (those arrays are double-buffered), so
// no second grid-wide step is needed between the update and the SpMV.
//
// Set-up: k_cg_init forms w_0 = M D^-1 r_0 and the partials of
// (gamma_0, delta_0, |r_0|^2).  Columns converge when |r|^2 <= rtol^2 |b|^2.

// w_0 = M D^-1 r_0 and partials (r.u, w.u, r.r).
__global__ __launch_bounds__(kWG) void k_cg_init(CgArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  const bool on = a.colK[c] >= a.kneed;
  double sums[3] = {0.0, 0.0, 0.0};
  if (on) {
    for (int e = L.row0; e < L.rend; e += L.rstride) {
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) {
        const int col = o.ell_col[5 * e + j];
        w += o.mass[5 * e + j] * (o.dinv[col] * a.r_in[(size_t)col * Bs + c]);
      }
      const size_t ie = (size_t)e * Bs + c;
      const double r = a.r_in[ie], u = o.dinv[e] * r;
      a.w_out[ie] = w;
      sums[0] += r * u;
      sums[1] += w * u;
      sums[2] += r * r;
    }
  }
  wg_partials<3>(L, sums, a.part_out, a.rb.max_wg);
}

// Fused small-batch prologue (Bs <= 4, tile 0, one wave per column): reduce
// the previous kernel's partials, test convergence, form alpha and beta.
// Workgroup 0 publishes the scalars into the iteration's parity slot; all
// workgroups take the same decisions from the same sums.
struct FusedCols {
  double alpha[4], beta[4];
  int act[4];
  int any;
};

__device__ void fused_step(const CgArgs &a, const Lane &L, FusedCols &fc) {
  const SolveState st = a.st;
  if (threadIdx.x == 0) fc.any = 0;
  __syncthreads();
  const int cc = L.wave;
  if (cc < L.ct) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int g = L.lane; g < a.nwg_prev; g += 64)
#pragma unroll
      for (int q = 0; q < 3; q++) v[q] += a.part_in[((size_t)g * 3 + q) * 64 + cc];
#pragma unroll
    for (int q = 0; q < 3; q++) v[q] = wave_col_sum(v[q], 1);
    if (L.lane == 0) {
      const int cur = a.k & 1, prev = cur ^ 1;
      const bool w0 = blockIdx.x == 0;
      double alpha = 0.0, beta = 0.0;
      int act = 0;
      if (a.k == 0) {
        act = (a.colK[cc] >= a.kneed && v[2] > 0.0) ? 1 : 0;
        alpha = act ? v[0] / v[1] : 0.0;
        if (w0) {
          st.bb[cc] = v[2];
          st.resid[cc] = act ? 1.0 : 0.0;
          st.it2[cur * 4 + cc] = 0;
          st.rz2[cur * 4 + cc] = v[0];
          st.al2[cur * 4 + cc] = alpha;
        }
      } else if (st.act2[prev * 4 + cc]) {
        const int it = st.it2[prev * 4 + cc] + 1;
        const double bb = st.bb[cc];
        bool fail = false;
        if (v[2] <= a.rtol2 * bb) {
          act = 0;
        } else if (it >= a.maxit) {
          fail = true;
        } else {
          act = 1;
          beta = v[0] / st.rz2[prev * 4 + cc];
          alpha = v[0] / (v[1] - beta * v[0] / st.al2[prev * 4 + cc]);
        }
        if (w0) {
          st.it2[cur * 4 + cc] = it;
          st.rz2[cur * 4 + cc] = v[0];
          st.al2[cur * 4 + cc] = alpha;
          st.resid[cc] = sqrt(v[2] / bb);
          if (fail) atomicAdd(st.fail, 1);
          if (act && a.last_check) atomicAdd(st.budget_fail, 1);
          atomicMax(st.iter_max, it);
        }
      }
      if (w0) st.act2[cur * 4 + cc] = act;
      fc.alpha[cc] = alpha;
      fc.beta[cc] = beta;
      fc.act[cc] = act;
      if (act) atomicOr(&fc.any, 1);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int n = 0;
    for (int j = 0; j < L.ct; j++) n += fc.act[j];
    st.cnt[a.k & 1] = n;
    if (a.count_cols && n > 0 && !a.check_only) {
      atomicAdd(&st.prof[0], (unsigned)n);
      atomicAdd(&st.prof[1], 1u);
    }
  }
}

// One CG iteration for every active column.
__global__ __launch_bounds__(kWG) void k_cg_iter(CgArgs a) {
  const SolveState st = a.st;
  const Lane L = lane_map(a.Bs, a.ops.ne);
  __shared__ FusedCols fc;
  bool act;
  double alpha, beta;
  if (a.fused) {
    fused_step(a, L, fc);
    if (!fc.any || a.check_only) return;
    act = fc.act[L.col] != 0;
    alpha = fc.alpha[L.col];
    beta = fc.beta[L.col];
  } else {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st.cnt[a.k & 1] = 0;
    if (st.cnt[(a.k + 1) & 1] == 0) return;
    if (a.count_cols) count_active(L, st);
    act = st.active[L.col] != 0;
    alpha = act ? st.alpha[L.col] : 0.0;
    beta = act ? st.beta[L.col] : 0.0;
  }
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  double sums[3] = {0.0, 0.0, 0.0};
  if (act) {
    for (int e = L.row0; e < L.rend; e += L.rstride) {
      double wn = 0.0, se = 0.0, rn = 0.0, un = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) {
        const int col = o.ell_col[5 * e + j];
        const size_t ij = (size_t)col * Bs + c;
        double s = a.w_in[ij];
        if (beta != 0.0) s += beta * a.s_in[ij];
        const double r = a.r_in[ij] - alpha * s;
        const double u = o.dinv[col] * r;
        wn += o.mass[5 * e + j] * u;
        if (j == 0) {
          se = s;
          rn = r;
          un = u;
        }
      }
      const size_t ie = (size_t)e * Bs + c;
      double p = o.dinv[e] * a.r_in[ie];
      if (beta != 0.0) p += beta * a.p[ie];
      a.p[ie] = p;
      a.x[ie] += alpha * p;
      a.s_out[ie] = se;
      a.r_out[ie] = rn;
      a.w_out[ie] = wn;
      sums[0] += rn * un;
      sums[1] += wn * un;
      sums[2] += rn * rn;
    }
  }
  wg_partials<3>(L, sums, a.part_out, a.rb.max_wg);
}

// ------------------------------------------- forward combination of a basis
// E[row][mem*G + m] = sum_k cf[k][m] R_k[row][mem], both row ranges, with
// t = row * BsR + mem.  A workgroup takes tiles of kTT consecutive t: it
// stages R_k[t] (k in chunks of kKC) and the matching coefficients in LDS;
// thread (tb, mb) = (tid % 16, tid / 16) forms the 4 x 4 block t = tb + 16 i,
// m = 4 mb + j (four consecutive outputs of a t leave as one run), so that
// each pair of LDS reads feeds two multiply-adds.  k runs in ascending order
// as in the definition.
constexpr int kTT = 64;  // t per tile
constexpr int kKC = 64;  // k (or m) per LDS chunk

__global__ __launch_bounds__(kWG) void k_combine(CombineArgs a) {
  __shared__ double bt[kKC][kTT];
  __shared__ double cs[kKC][64];
  const int tb = threadIdx.x & 15, mb = threadIdx.x >> 4;
  const long total = (long)a.nrows * a.BsR;
  const long ntiles = (total + kTT - 1) / kTT;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long t0 = tile * kTT;
    const int nt = (int)min((long)kTT, total - t0);
    for (int mc = 0; mc < a.G; mc += 64) {
      double acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.0;
      for (int k0 = 0; k0 <= a.kmax; k0 += kKC) {
        const int nk = min(kKC, a.kmax + 1 - k0);
        // staging: every load of the chunk issued before the first LDS store
        double vb[kKC * kTT / kWG], vc[kKC * 64 / kWG];
#pragma unroll
        for (int r = 0; r < kKC * kTT / kWG; r++) {
          const int idx = threadIdx.x + r * kWG, kk = idx / kTT, i = idx % kTT;
          vb[r] = kk < nk && i < nt ? a.basis[(size_t)(k0 + kk) * a.basis_stride + t0 + i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kKC * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG, kk = idx / 64, j = idx % 64;
          vc[r] = kk < nk && mc + j < a.G ? a.cf[(size_t)(k0 + kk) * a.G + mc + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kKC * kTT / kWG; r++) {
          const int idx = threadIdx.x + r * kWG;
          bt[idx / kTT][idx % kTT] = vb[r];
        }
#pragma unroll
        for (int r = 0; r < kKC * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG;
          cs[idx / 64][idx % 64] = vc[r];
        }
        __syncthreads();
        for (int kk = 0; kk < nk; kk++) {
          double b[4], c[4];
#pragma unroll
          for (int i = 0; i < 4; i++) b[i] = bt[kk][tb + 16 * i];
#pragma unroll
          for (int j = 0; j < 4; j++) c[j] = cs[kk][4 * mb + j];
#pragma unroll
          for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = fma(c[j], b[i], acc[i][j]);
        }
      }
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int ti = tb + 16 * i;
        if (ti < nt) {
          const long t = t0 + ti;
          const bool on = (int)(t % a.BsR) < a.members;
#pragma unroll
          for (int j = 0; j < 4; j++) {
            const int m = mc + 4 * mb + j;
            if (m < a.G) a.E[t * a.G + m] = on ? acc[i][j] : 0.0;
          }
        }
      }
    }
  }
}

// Single-chunk forms of k_combine and k_reduce_terms (Kmax < kKC, G <= 64,
// the usual shapes), on the matrix cores: both are dense contractions over
// a tile of 64 values of t, done as 16 x 16 x 4 FP64 MFMA blocks (each
// operand value read once from LDS per block instead of once per
// multiply-add).  The coefficients are staged once per workgroup, and each
// workgroup walks its tiles with the next tile's loads in flight during the
// current tile's arithmetic.  Lane layout of v_mfma_f64_16x16x4f64 (lane l):
// A[l % 16][l / 16], B[l / 16][l % 16], result register r holds
// D[4 r + l / 16][l % 16].  The sums run over k (or m) in blocks of four.
typedef double d4v __attribute__((ext_vector_type(4)));

// E[t][m] = sum_k R_k[t] cf[k][m]: wave w takes t0 + 16 w .. + 15 and all
// four 16-column blocks of m.
__global__ __launch_bounds__(kWG) void k_combine1(CombineArgs a) {
  __shared__ double bt[kKC][kTT];
  __shared__ double cs[kKC][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long total = (long)a.nrows * a.BsR;
  const long ntiles = (total + kTT - 1) / kTT;
  const int nk = a.kmax + 1;
  for (int idx = threadIdx.x; idx < kKC * 64; idx += kWG) {
    const int kk = idx / 64, j = idx % 64;
    cs[kk][j] = kk < nk && j < a.G ? a.cf[(size_t)kk * a.G + j] : 0.0;
  }
  double vb[kKC * kTT / kWG];
  auto fetch = [&](long tile) {
    const long t0 = tile * kTT;
#pragma unroll
    for (int r = 0; r < kKC * kTT / kWG; r++) {
      const int idx = threadIdx.x + r * kWG, kk = idx / kTT, i = idx % kTT;
      vb[r] = tile < ntiles && kk < nk && t0 + i < total ? a.basis[(size_t)kk * a.basis_stride + t0 + i] : 0.0;
    }
  };
  fetch(blockIdx.x);
  const int nk4 = (nk + 3) & ~3;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long t0 = tile * kTT;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKC * kTT / kWG; r++) {
      const int idx = threadIdx.x + r * kWG;
      bt[idx / kTT][idx % kTT] = vb[r];
    }
    __syncthreads();
    fetch(tile + gridDim.x);
    d4v acc[4];
#pragma unroll
    for (int mb = 0; mb < 4; mb++) acc[mb] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < nk4; k0 += 4) {
      const double av = bt[k0 + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < 4; mb++)
        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, cs[k0 + (lane >> 4)][16 * mb + (lane & 15)], acc[mb], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const long t = t0 + 16 * w + 4 * r + (lane >> 4);
      if (t < total) {
        const bool on = (int)(t % a.BsR) < a.members;
#pragma unroll
        for (int mb = 0; mb < 4; mb++) {
          const int m = 16 * mb + (lane & 15);
          if (m < a.G) a.E[t * a.G + m] = on ? acc[mb][r] : 0.0;
        }
      }
    }
  }
}

// Z[k][t] = sum_m cb[k][m] Y[t][m]: wave w takes t0 + 16 w .. + 15 and all
// 16-row blocks of k (D^T = cb Y^T, so that each result row of k leaves as
// 16 consecutive values of t).
__global__ __launch_bounds__(kWG) void k_reduce_terms1(ReduceTermsArgs a) {
  __shared__ double ys[kTT][65];
  __shared__ double cs[kKC][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long total = (long)a.nrows * a.BsZ;
  const long ntiles = (total + kTT - 1) / kTT;
  const int nk = a.kmax + 1, nm = a.G;
  for (int idx = threadIdx.x; idx < kKC * 64; idx += kWG) {
    const int kk = idx / 64, j = idx % 64;
    cs[kk][j] = kk < nk && j < nm ? a.cb[(size_t)kk * a.G + j] : 0.0;
  }
  double vy[kTT * 64 / kWG];
  auto fetch = [&](long tile) {
    const long t0 = tile * kTT;
#pragma unroll
    for (int r = 0; r < kTT * 64 / kWG; r++) {
      const int idx = threadIdx.x + r * kWG, i = idx / 64, j = idx % 64;
      vy[r] = tile < ntiles && t0 + i < total && j < nm ? a.Y[(t0 + i) * a.G + j] : 0.0;
    }
  };
  fetch(blockIdx.x);
  const int nm4 = (nm + 3) & ~3;
  const int nkb = (nk + 15) >> 4;  // 16-row blocks of k (at most 4)
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long t0 = tile * kTT;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTT * 64 / kWG; r++) {
      const int idx = threadIdx.x + r * kWG;
      ys[idx / 64][idx % 64] = vy[r];
    }
    __syncthreads();
    fetch(tile + gridDim.x);
    d4v acc[4];
#pragma unroll
    for (int kb = 0; kb < 4; kb++) acc[kb] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < nm4; m0 += 4) {
      const double bv = ys[16 * w + (lane & 15)][m0 + (lane >> 4)];
#pragma unroll
      for (int kb = 0; kb < 4; kb++)
        if (kb < nkb)
          acc[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cs[16 * kb + (lane & 15)][m0 + (lane >> 4)], bv, acc[kb], 0, 0, 0);
    }
#pragma unroll
    for (int kb = 0; kb < 4; kb++)
      if (kb < nkb) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int k = 16 * kb + 4 * r + (lane >> 4);
          const long t = t0 + 16 * w + (lane & 15);
          if (k < nk && t < total) a.Z[(size_t)k * a.zstride + t] = acc[kb][r];
        }
      }
  }
}

// Z[k][t] = sum_m cb[k][m] Y[t][m] (backward terms reduced to one series per
// member).  A workgroup stages kTT rows Y[t][.] (m in chunks of 64) and cb
// for a chunk of kKC values of k in LDS, both padded to 65 doubles a row
// against bank conflicts; thread (tb, kb) = (tid % 16, tid / 16) forms the
// 4 x 4 block t = tb + 16 i, k = k0 + kb + 16 j, so that each pair of LDS
// reads feeds two multiply-adds.  m runs in ascending order.
__global__ __launch_bounds__(kWG) void k_reduce_terms(ReduceTermsArgs a) {
  __shared__ double ys[kTT][65];
  __shared__ double cs[kKC][65];
  const int tb = threadIdx.x & 15, kb = threadIdx.x >> 4;
  const long total = (long)a.nrows * a.BsZ;
  const long ntiles = (total + kTT - 1) / kTT;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long t0 = tile * kTT;
    const int nt = (int)min((long)kTT, total - t0);
    for (int k0 = 0; k0 <= a.kmax; k0 += kKC) {
      const int nk = min(kKC, a.kmax + 1 - k0);
      double acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.0;
      for (int mc = 0; mc < a.G; mc += 64) {
        const int nm = min(64, a.G - mc);
        // staging: every load of the chunk issued before the first LDS store
        double vy[kTT * 64 / kWG], vc[kKC * 64 / kWG];
#pragma unroll
        for (int r = 0; r < kTT * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG, i = idx / 64, j = idx % 64;
          vy[r] = i < nt && j < nm ? a.Y[(t0 + i) * a.G + mc + j] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kKC * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG, kk = idx / 64, j = idx % 64;
          vc[r] = kk < nk && j < nm ? a.cb[(size_t)(k0 + kk) * a.G + mc + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kTT * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG;
          ys[idx / 64][idx % 64] = vy[r];
        }
#pragma unroll
        for (int r = 0; r < kKC * 64 / kWG; r++) {
          const int idx = threadIdx.x + r * kWG;
          cs[idx / 64][idx % 64] = vc[r];
        }
        __syncthreads();
        for (int m = 0; m < nm; m++) {
          double y[4], c[4];
#pragma unroll
          for (int i = 0; i < 4; i++) y[i] = ys[tb + 16 * i][m];
#pragma unroll
          for (int j = 0; j < 4; j++) c[j] = cs[kb + 16 * j][m];
#pragma unroll
          for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = fma(c[j], y[i], acc[i][j]);
        }
      }
#pragma unroll
      for (int j = 0; j < 4; j++)
        if (kb + 16 * j < nk) {
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (tb + 16 * i < nt) a.Z[(size_t)(k0 + kb + 16 * j) * a.zstride + t0 + tb + 16 * i] = acc[i][j];
        }
    }
  }
}

// ----------------------------------------------------------- nonlinearity

// Per cell and local edge i, the cell's share of the velocity right-hand side
// of test function phi_i, and the depth tendency:
//   C_i = |T| u(xbar) . grad^perp q_i + (s_i/|T|) int |u|^2/2
//         - sum_a s_a int_{side a} (t_e . u~) q_i ds,
//   q_i = (k x u) . phi_i (affine on T), eta2 = -sum_a s_a U_a (eta-b)_up / |T|.
// Everything but the upwind traces u~ is fixed by the cell's geometry, so the
// operators carry C_i as forms in the cell's edge fluxes U (nlform: a
// symmetric 3x3 form per i for the volume and kinetic-energy terms, and per
// side and Gauss point the coefficients of U in q_i); the kernel evaluates
// the forms (about 120 FP64 operations per cell and column).
// UNI (blocks of at least 64 columns): a wave works on one cell, so the cell
// index is made wave-uniform and the cell's tables are the same for the
// whole wave.
template <bool UNI>
__global__ __launch_bounds__(kWG) void k_nl_cell(NlArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.nc);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  for (int tl = L.row0; tl < L.rend; tl += L.rstride) {
    const int t = UNI ? __builtin_amdgcn_readfirstlane(tl) : tl;
    // the cell's edges and its neighbours' edges: one 48-byte record,
    // loaded whole (12 edge numbers)
    int s[3], ed[12], nb[3];
    double F[kNlForm], bt, bn[3], ia;
    if (UNI) {
      // the cell's tables, the same for the whole wave: scalar loads
      const auto *rec = uniform_ro(o.cell_edges) + 12 * (size_t)t;
#pragma unroll
      for (int j = 0; j < 12; j++) ed[j] = rec[j];
      const auto *fr = uniform_ro(o.nlform) + (size_t)kNlForm * t;
#pragma unroll
      for (int j = 0; j < kNlForm; j++) F[j] = fr[j];
#pragma unroll
      for (int j = 0; j < 3; j++) {
        s[j] = uniform_ro(o.csgn)[3 * t + j];
        nb[j] = uniform_ro(o.cnbr)[3 * t + j];
        bn[j] = uniform_ro(o.bottom)[nb[j]];
      }
      bt = uniform_ro(o.bottom)[t];
      ia = uniform_ro(o.inv_area)[t];
    } else {
      const int4 *rec = reinterpret_cast<const int4 *>(o.cell_edges) + 3 * (size_t)t;
      const int4 q0 = rec[0], q1 = rec[1], q2 = rec[2];
      ed[0] = q0.x; ed[1] = q0.y; ed[2] = q0.z; ed[3] = q0.w;
      ed[4] = q1.x; ed[5] = q1.y; ed[6] = q1.z; ed[7] = q1.w;
      ed[8] = q2.x; ed[9] = q2.y; ed[10] = q2.z; ed[11] = q2.w;
      const double *fr = o.nlform + (size_t)kNlForm * t;
#pragma unroll
      for (int j = 0; j < kNlForm; j++) F[j] = fr[j];
#pragma unroll
      for (int j = 0; j < 3; j++) {
        s[j] = o.csgn[3 * t + j];
        nb[j] = o.cnbr[3 * t + j];
        bn[j] = o.bottom[nb[j]];
      }
      bt = o.bottom[t];
      ia = o.inv_area[t];
    }
    double U[3];
#pragma unroll
    for (int j = 0; j < 3; j++) U[j] = a.u[(size_t)ed[j] * Bs + c];
    // volume and kinetic-energy terms: U^T S_i U
    const double P[6] = {U[0] * U[0], U[1] * U[1], U[2] * U[2], U[0] * U[1], U[0] * U[2], U[1] * U[2]};
    double Cv[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double v = F[6 * i] * P[0];
#pragma unroll
      for (int m = 1; m < 6; m++) v = fma(F[6 * i + m], P[m], v);
      Cv[i] = v;
    }
    // facet terms, side by side: the upwind tangential velocity at the
    // side's two Gauss points, from the cell the edge flux leaves (flux > 0:
    // the edge's first cell, otherwise its second), that cell's three edges
    // against the edge's trace table.  This cell is the edge's first cell
    // exactly when s = +1, so the upwind cell is this one when the flux and s
    // have the same sign, else the neighbour across the side.  The upwind
    // cell's edges and table are chosen per column as row numbers and
    // offsets, so that every column loads (no branch around the loads).
    double uu[3][3];
    const double *tau[3];
#pragma unroll
    for (int aa = 0; aa < 3; aa++) {
      const int sid = s[aa] > 0 ? 0 : 1;  // this cell's place in the edge's cell pair
      const bool self_up = (U[aa] > 0.0) == (s[aa] > 0);
      tau[aa] = o.tau + (size_t)kEdgeTau * ed[aa] + 6 * (self_up ? sid : 1 - sid);
#pragma unroll
      for (int j = 0; j < 3; j++) uu[aa][j] = a.u[(size_t)(self_up ? ed[j] : ed[3 + 3 * aa + j]) * Bs + c];
    }
#pragma unroll
    for (int aa = 0; aa < 3; aa++) {
#pragma unroll
      for (int gp = 0; gp < 2; gp++) {
        double utg = tau[aa][3 * gp] * uu[aa][0];
        utg = fma(tau[aa][3 * gp + 1], uu[aa][1], utg);
        utg = fma(tau[aa][3 * gp + 2], uu[aa][2], utg);
        const double *H = F + 18 + (2 * aa + gp) * 9;
#pragma unroll
        for (int i = 0; i < 3; i++) {
          double q = H[3 * i] * U[0];
          q = fma(H[3 * i + 1], U[1], q);
          q = fma(H[3 * i + 2], U[2], q);
          Cv[i] = fma(utg, q, Cv[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 3; i++) a.C[((size_t)3 * t + i) * Bs + c] = Cv[i];
    // depth: upwind (eta - b) on every side (this cell or the neighbour,
    // chosen per column as a row number as above)
    const size_t it = (size_t)t * Bs + c;
    double r = 0.0;
#pragma unroll
    for (int aa = 0; aa < 3; aa++) {
      const bool self_up = (U[aa] > 0.0) == (s[aa] > 0);
      const int cu = self_up ? t : nb[aa];
      const double hv = a.eta[(size_t)cu * Bs + c] - (self_up ? bt : bn[aa]);
      r -= s[aa] * U[aa] * hv;
    }
    a.out_eta[it] = r * ia;
  }
}

// Velocity right-hand side r_e = C[c0][l0] + C[c1][l1] and CG start x = 0.
template <bool UNI>
__global__ __launch_bounds__(kWG) void k_nl_gather(GatherArgs a) {
  folded_check(a.chk, a.chk_blocks);
  const Lane L = lane_map(a.Bs, a.ops.ne);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  double rr = 0.0;
  if (a.colK[c] >= a.kneed) {
    for (int el = L.row0; el < L.rend; el += L.rstride) {
      const int e = urow<UNI>(el);
      const size_t ie = (size_t)e * Bs + c;
      const double r = a.C[(size_t)rl<UNI>(o.cidx, 2 * e) * Bs + c] + a.C[(size_t)rl<UNI>(o.cidx, 2 * e + 1) * Bs + c];
      a.r[ie] = r;
      if (!a.r32) a.x[ie] = 0.0;  // the refined solve's first refinement writes x
      if (a.d0) a.d0[ie] = a.theta_inv * rl<UNI>(o.dinv, e) * r;
      if (a.r32) {
        const float r32 = (float)r;
        a.r32[ie] = r32;
        a.x1_32[ie] = a.theta_inv32 * rl<UNI>(o.dinv32, e) * r32;
      }
      if (a.part_rr) rr += r * r;
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) a.st.cnt[1] = 0;
  if (a.part_rr) {
    double v[1] = {rr};
    wg_partials<1>(L, v, a.part_rr, a.max_wg);
  }
}

// ----------------------------------------------------------- elementwise
// acc[row][c/G] += sum over the G-column group of coef[c] * in[row][c]
// (columns with colK[c] >= acc_k), over both row ranges.
__global__ __launch_bounds__(kWG) void k_acc(AccArgs a) {
  const Lane L = lane_map(a.Bs, a.nrows);
  const int c = L.col, Bs = a.Bs;
  const bool on = a.colK[c] >= a.acc_k;
  const double coef = on ? a.coef[c] : 0.0;
  for (int base = L.row0 - L.lane / L.ct; base < L.rend; base += L.rstride) {
    const int row = base + L.lane / L.ct;
    const bool in = row < L.rend;
    double v = (in && on) ? coef * a.in[(size_t)row * Bs + c] : 0.0;
    v = lane_group_sum(v, a.G);
    if (in && (c % a.G) == 0) a.acc[(size_t)row * (Bs / a.G) + c / a.G] += v;
  }
}

// out[i] = a0 x0[i] + a1 x1[i] + a2 x2[i] (null inputs skipped).
__global__ __launch_bounds__(kWG) void k_axpy(AxpyArgs a) {
  for (size_t i = (size_t)blockIdx.x * kWG + threadIdx.x; i < a.n; i += (size_t)gridDim.x * kWG) {
    double v = 0.0;
    if (a.x0) v += a.a0 * a.x0[i];
    if (a.x1) v += a.a1 * a.x1[i];
    if (a.x2) v += a.a2 * a.x2[i];
    a.out[i] = v;
  }
}

// Member-major states [B][n] <-> block [row][Bs] (u rows then eta rows).
__global__ __launch_bounds__(kWG) void k_to_block(TransArgs a) {
  const size_t total = (size_t)a.n * a.Bs;
  for (size_t i = (size_t)blockIdx.x * kWG + threadIdx.x; i < total; i += (size_t)gridDim.x * kWG) {
    const int row = (int)(i / a.Bs), c = (int)(i % a.Bs);
    a.blk[i] = c < a.B ? a.states[(size_t)c * a.n + row] : 0.0;
  }
}
__global__ __launch_bounds__(kWG) void k_from_block(TransArgs a) {
  const size_t total = (size_t)a.n * a.B;
  for (size_t i = (size_t)blockIdx.x * kWG + threadIdx.x; i < total; i += (size_t)gridDim.x * kWG) {
    const int c = (int)(i / a.n), row = (int)(i % a.n);
    a.states[i] = a.blk[(size_t)row * a.Bs + c];
  }
}

// Per-column diagnostics, reduced deterministically (finalize FIN_OUT):
//   q0 = u' M u, q1 = sum |c| eta, q2 = sum |c| eta^2, q3 = sum (D u)^2 / |c|,
//   q4 = sum_c (H + eta - b) int_c |u|^2 / 2   (RT0 velocity, side midpoints).
__global__ __launch_bounds__(kWG) void k_diag(DiagArgs a) {
  const Lane L = lane_map(a.Bs, a.ops.ne > a.ops.nc ? a.ops.ne : a.ops.nc);
  const DevOps &o = a.ops;
  const int c = L.col, Bs = a.Bs;
  double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int r = L.row0; r < L.rend; r += L.rstride) {
    if (r < o.ne) {
      double mu = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) mu += o.mass[5 * r + j] * a.u[(size_t)o.ell_col[5 * r + j] * Bs + c];
      sums[0] += a.u[(size_t)r * Bs + c] * mu;
    }
    if (r < o.nc) {
      const double A = o.area[r], eta = a.eta[(size_t)r * Bs + c];
      sums[1] += A * eta;
      sums[2] += A * eta * eta;
      const double *g = o.cgeo + (size_t)r * kCellGeo;
      double U[3], div = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        U[j] = o.csgn[3 * r + j] * a.u[(size_t)o.cedge[3 * r + j] * Bs + c];
        div += U[j];
      }
      sums[3] += div * div / A;
      double ke = 0.0;
#pragma unroll
      for (int q = 0; q < 3; q++) {
        double u2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++) {
          const double x = 0.5 * (g[3 * ((q + 1) % 3) + d] + g[3 * ((q + 2) % 3) + d]);
          double v = 0.0;
#pragma unroll
          for (int j = 0; j < 3; j++) v += U[j] * (x - g[3 * j + d]);
          v *= 0.5 / A;
          u2 += v * v;
        }
        ke += (A / 3.0) * 0.5 * u2;
      }
      sums[4] += (a.H + eta - o.bottom[r]) * ke;
    }
  }
  wg_partials<5>(L, sums, a.part, a.max_wg);
}

// Clear small integer/double buffers (used instead of memset so that the
// sequence stays capturable).
__global__ void k_zero(unsigned *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// ------------------------------------------------------------- finalize
// Column sums of the per-workgroup partials of the preceding kernel, one
// wave per column (lane j adds partials j, j+64, ...; then a fixed shuffle
// tree), followed by the per-column update of the CG scalars:
//   FIN_INIT  bb = r.r, rz = r.z, active = colK >= kneed && bb > 0
//   FIN_ALPHA alpha = rz / p.q
//   FIN_BETA  convergence test ||r||^2 <= rtol^2 bb, else beta = rz'/rz
//   FIN_OUT   plain sums to out[q * Bs + c]
// Active columns are counted into cnt[slot_out] (integer atomics).
__global__ __launch_bounds__(kWG) void k_finalize(FinArgs a) {
  const SolveState st = a.st;
  if (a.mode == FIN_STEP && st.cnt[a.slot_in] == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ct = a.Bs < 64 ? a.Bs : 64;
  const int cpb = ct < 4 ? ct : 4;            // columns per workgroup
  const int blocks_per_tile = ct / cpb;
  const int tile = blockIdx.x / blocks_per_tile;
  const int cl = (blockIdx.x % blocks_per_tile) * cpb + wave;  // column in tile
  if (wave >= cpb) return;
  const int c = tile * ct + cl;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int w = lane; w < a.nwg; w += 64)
    for (int q = 0; q < a.nq; q++)
      v[q] += a.part[(((size_t)tile * a.max_wg + w) * a.nq + q) * 64 + cl];
  for (int q = 0; q < a.nq; q++) v[q] = wave_col_sum(v[q], 1);
  if (lane != 0) return;
  bool on = false;
  if (a.mode == FIN_INIT) {
    // (gamma_0, delta_0, |b|^2)
    on = a.colK[c] >= a.kneed && v[2] > 0.0;
    st.bb[c] = v[2];
    st.rz[c] = v[0];
    st.alpha[c] = on ? v[0] / v[1] : 0.0;
    st.beta[c] = 0.0;
    st.iters[c] = 0;
    st.resid[c] = on ? 1.0 : 0.0;
    st.active[c] = on ? 1 : 0;
  } else if (a.mode == FIN_STEP) {
    // (gamma', delta', |r'|^2) after one iteration
    if (st.active[c]) {
      const int it = st.iters[c] + 1;
      st.iters[c] = it;
      st.resid[c] = sqrt(v[2] / st.bb[c]);
      if (v[2] <= a.rtol2 * st.bb[c]) {
        st.active[c] = 0;
      } else if (it >= a.maxit) {
        st.active[c] = 0;
        atomicAdd(st.fail, 1);
      } else {
        const double beta = v[0] / st.rz[c];
        st.alpha[c] = v[0] / (v[1] - beta * v[0] / st.alpha[c]);
        st.beta[c] = beta;
        st.rz[c] = v[0];
        on = true;
        if (a.last_check) atomicAdd(st.budget_fail, 1);
      }
      atomicMax(st.iter_max, it);
    }
  } else {
    for (int q = 0; q < a.nq; q++) a.out[q * a.Bs + c] = v[q];
  }
  if (on) atomicAdd(&st.cnt[a.slot_out], 1);
}

// ------------------------------------------------------------ launchers
namespace {
// Workgroups along the rows of one column tile (a multiple of 8, see
// lane_map).  Narrow batches (Bs <= 4) are latency-bound: about four rows per
// thread keeps the launch short and the partial sums few.  Wider ones fill
// the 256 CUs several times over, split over the column tiles.
// process default launch shape (pa_set_launch_tune), and the shape of the
// call the calling thread is enqueueing (TuneScope)
LaunchTune g_default_tune;
std::mutex g_default_mu;
thread_local const LaunchTune *t_tune = nullptr;
// measurement hook: events that the next launch of a profiled kernel
// records as part of its dispatch (start and end of the kernel itself)
hipEvent_t g_ev0 = nullptr, g_ev1 = nullptr;

template <typename K, typename A>
void launch_timed(K kernel, dim3 grid, hipStream_t s, const A &a) {
  if (g_ev0) {
    hipExtLaunchKernelGGL(kernel, grid, dim3(kWG), 0, s, g_ev0, g_ev1, 0, a);
    g_ev0 = g_ev1 = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, dim3(kWG), 0, s, a);
  }
}

int grid_rows(int rows, int Bs) {
  const int ct = Bs < 64 ? Bs : 64;
  const int rows_per_pass = (kWG / 64) * (64 / ct);
  const int ctiles = (Bs + 63) / 64;
  int want, cap;
  const LaunchTune tune = launch_tuning();
  if (Bs <= 4) {
    const int rpt = tune.narrow_rows_per_thread;
    want = (rows + rpt * rows_per_pass - 1) / (rpt * rows_per_pass);
    cap = 2048;
  } else {
    want = (rows + rows_per_pass - 1) / rows_per_pass;
    cap = ctiles >= 8 ? 256 : tune.wide_max_wg / ctiles;
  }
  int g = want < cap ? want : cap;
  g = (g + 7) / 8 * 8;
  return g > 0 ? g : 8;
}
int grid_flat(size_t n) {
  size_t g = (n + kWG - 1) / kWG;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}
// workgroups of the tile kernels (kTT values of t per tile), grid-stride
// beyond 2048
int grid_tiles(size_t n) {
  const size_t g = (n + kTT - 1) / kTT;
  return (int)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}
// the pipelined single-chunk forms: two workgroups per CU, each walking
// several tiles
int grid_tiles_pipe(size_t n) {
  const size_t g = (n + kTT - 1) / kTT;
  return (int)(g < 512 ? (g > 0 ? g : 1) : 512);
}
dim3 rows_grid(int rows, int Bs) { return dim3(grid_rows(rows, Bs), (Bs + 63) / 64); }
// One pass over the rows, a row (and up to 64 columns) a wave: for kernels
// that keep no per-workgroup partials and whose rows each wait on dependent
// gathers (the cell kernel of N), so that as many rows as fit are in flight.
dim3 rows_grid_full(int rows, int Bs) {
  const int ct = Bs < 64 ? Bs : 64;
  const int rows_per_pass = (kWG / 64) * (64 / ct);
  int g = (rows + rows_per_pass - 1) / rows_per_pass;
  g = (g + 7) / 8 * 8;
  return dim3(g > 0 ? g : 8, (Bs + 63) / 64);
}
}  // namespace

int launch_max_wg() { return 2048; }
LaunchTune launch_default() {
  std::lock_guard<std::mutex> lk(g_default_mu);
  return g_default_tune;
}
void set_launch_default(const LaunchTune &t) {
  std::lock_guard<std::mutex> lk(g_default_mu);
  g_default_tune = clamp_tune(t);
}
LaunchTune launch_tuning() { return t_tune ? *t_tune : launch_default(); }
LaunchTune clamp_tune(LaunchTune t) {
  if (t.narrow_rows_per_thread < 1) t.narrow_rows_per_thread = 1;
  if (t.wide_max_wg < 8) t.wide_max_wg = 8;
  if (t.wide_max_wg > 2048) t.wide_max_wg = 2048;
  if (t.lp_min_cols < 1) t.lp_min_cols = 1;
  if (t.mixed_min_cols < 1) t.mixed_min_cols = 1;
  if (t.fused_steps < 1) t.fused_steps = 1;
  if (t.fused_steps > kFusedMax) t.fused_steps = kFusedMax;
  return t;
}
TuneScope::TuneScope(const LaunchTune &t) : prev_(t_tune) { t_tune = &t; }
TuneScope::~TuneScope() { t_tune = prev_; }
int launch_rows_grid(int rows, int Bs) { return grid_rows(rows, Bs); }

void launch_stiff(const StiffArgs &a, hipStream_t s) {
  const int nrow = a.ops.ne > a.ops.nc ? a.ops.ne : a.ops.nc;
  if (a.Bs >= 64)
    hipLaunchKernelGGL(k_stiff<true>, rows_grid(nrow, a.Bs), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_stiff<false>, rows_grid(nrow, a.Bs), dim3(kWG), 0, s, a);
}
void launch_cg_init(const CgArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
}
void arm_launch_events(hipEvent_t e0, hipEvent_t e1) {
  g_ev0 = e0;
  g_ev1 = e1;
}
bool launch_events_armed() { return g_ev0 != nullptr; }
void launch_cheb_iter(const ChebArgs &a, hipStream_t s) {
  launch_timed(k_cheb_iter, rows_grid(a.ops.ne, a.Bs), s, a);
}
void launch_cheb3_iter(const Cheb3Args &a, hipStream_t s) {
  if (a.Bs >= 64)
    hipLaunchKernelGGL(k_cheb3_iter<true>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_cheb3_iter<false>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
}
int cheb_fused_grid(const DevOps &o, int extra) {
  if (o.hparts <= 0 || o.fused_max < 2) return 0;
  const int g = (o.hparts + extra + 7) / 8 * 8;
  return g <= launch_max_wg() ? g : 0;
}
void launch_cheb_fused(const ChebFusedArgs &a, hipStream_t s) {
  const dim3 grid(cheb_fused_grid(a.ops, a.setup ? a.chk_blocks : 0));
  if (a.setup) {
    switch (a.slots[0]) {
      case 0: hipLaunchKernelGGL((k_cheb_fused<0, true>), grid, dim3(kFWG), 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_cheb_fused<1, true>), grid, dim3(kFWG), 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_cheb_fused<2, true>), grid, dim3(kFWG), 0, s, a); break;
      default: hipLaunchKernelGGL((k_cheb_fused<kRingSlots, true>), grid, dim3(kFWG), 0, s, a); break;
    }
    return;
  }
  switch (a.slots[0]) {
    case 0: hipLaunchKernelGGL((k_cheb_fused<0, false>), grid, dim3(kFWG), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_cheb_fused<1, false>), grid, dim3(kFWG), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_cheb_fused<2, false>), grid, dim3(kFWG), 0, s, a); break;
    default: hipLaunchKernelGGL((k_cheb_fused<kRingSlots, false>), grid, dim3(kFWG), 0, s, a); break;
  }
}
// The icosahedral meshes give P and P M widths 13 and 27 at every level;
// other widths take the generic loop.
void launch_cheb_lp_iter(const ChebLpArgs &a, hipStream_t s) {
  const bool fixed = a.lp.wp == 13 && a.lp.wpm == 27, uni = a.Bs >= 64;
  const dim3 g = rows_grid(a.ops.ne, a.Bs);
  if (fixed && uni)
    launch_timed(k_cheb_lp_iter<13, 27, true>, g, s, a);
  else if (fixed)
    launch_timed(k_cheb_lp_iter<13, 27, false>, g, s, a);
  else if (uni)
    launch_timed(k_cheb_lp_iter<0, 0, true>, g, s, a);
  else
    launch_timed(k_cheb_lp_iter<0, 0, false>, g, s, a);
}
void launch_lp_dir(const LpDirArgs &a, hipStream_t s) {
  const bool uni = a.Bs >= 64;
  const dim3 g = rows_grid(a.ops.ne, a.Bs);
  if (a.lp.wp == 13 && uni)
    launch_timed(k_lp_dir<13, true>, g, s, a);
  else if (a.lp.wp == 13)
    launch_timed(k_lp_dir<13, false>, g, s, a);
  else if (uni)
    launch_timed(k_lp_dir<0, true>, g, s, a);
  else
    launch_timed(k_lp_dir<0, false>, g, s, a);
}
int cheb_check_blocks(const CheckArgs &a) {
  const int ct = a.Bs < 64 ? a.Bs : 64;
  const int cpb = ct < 4 ? ct : 4;
  return ((a.Bs + 63) / 64) * (ct / cpb);
}
void launch_cheb_check(const CheckArgs &a, hipStream_t s) {
  const int ct = a.Bs < 64 ? a.Bs : 64;
  const int cpb = ct < 4 ? ct : 4;
  const int tiles = (a.Bs + 63) / 64;
  hipLaunchKernelGGL(k_cheb_check, dim3(tiles * (ct / cpb)), dim3(kWG), 0, s, a);
}
void launch_cheb32_iter(const Cheb32Args &a, hipStream_t s) {
  // the row mapping needs a power-of-two width up to 64, or a multiple of 64
  const int bq = a.Bs / 4;
  if (a.Bs >= 8 && a.Bs % 4 == 0 && ((bq & (bq - 1)) == 0 || bq % 64 == 0))
    if (a.Bs / 4 >= 64)
      hipLaunchKernelGGL(k_cheb32_iter4<true>, rows_grid(a.ops.ne, a.Bs / 4), dim3(kWG), 0, s, a);
    else
      hipLaunchKernelGGL(k_cheb32_iter4<false>, rows_grid(a.ops.ne, a.Bs / 4), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_cheb32_iter, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
}
void launch_refine(const RefineArgs &a, hipStream_t s) {
  if (a.Bs >= 64)
    hipLaunchKernelGGL(k_refine<true>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_refine<false>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
}
void launch_cg_iter(const CgArgs &a, hipStream_t s) {
  launch_timed(k_cg_iter, rows_grid(a.ops.ne, a.Bs), s, a);
}
void launch_combine(const CombineArgs &a, hipStream_t s) {
  if (a.kmax < kKC && a.G <= 64)
    hipLaunchKernelGGL(k_combine1, dim3(grid_tiles_pipe((size_t)a.nrows * a.BsR)), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_combine, dim3(grid_tiles((size_t)a.nrows * a.BsR)), dim3(kWG), 0, s, a);
}
void launch_reduce_terms(const ReduceTermsArgs &a, hipStream_t s) {
  if (a.kmax < kKC && a.G <= 64)
    hipLaunchKernelGGL(k_reduce_terms1, dim3(grid_tiles_pipe((size_t)a.nrows * a.BsZ)), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_reduce_terms, dim3(grid_tiles((size_t)a.nrows * a.BsZ)), dim3(kWG), 0, s, a);
}
void launch_nl_cell(const NlArgs &a, hipStream_t s) {
  if (a.Bs >= 64)
    hipLaunchKernelGGL(k_nl_cell<true>, rows_grid_full(a.ops.nc, a.Bs), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_nl_cell<false>, rows_grid_full(a.ops.nc, a.Bs), dim3(kWG), 0, s, a);
}
void launch_nl_gather(const GatherArgs &a, hipStream_t s) {
  if (a.Bs >= 64)
    hipLaunchKernelGGL(k_nl_gather<true>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL(k_nl_gather<false>, rows_grid(a.ops.ne, a.Bs), dim3(kWG), 0, s, a);
}
void launch_acc(const AccArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_acc, rows_grid(a.nrows, a.Bs), dim3(kWG), 0, s, a);
}
void launch_axpy(const AxpyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_flat(a.n)), dim3(kWG), 0, s, a);
}
void launch_to_block(const TransArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_to_block, dim3(grid_flat((size_t)a.n * a.Bs)), dim3(kWG), 0, s, a);
}
void launch_from_block(const TransArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_from_block, dim3(grid_flat((size_t)a.n * a.B)), dim3(kWG), 0, s, a);
}
void launch_diag(const DiagArgs &a, hipStream_t s) {
  const int nrow = a.ops.ne > a.ops.nc ? a.ops.ne : a.ops.nc;
  hipLaunchKernelGGL(k_diag, rows_grid(nrow, a.Bs), dim3(kWG), 0, s, a);
}
void launch_finalize(const FinArgs &a, hipStream_t s) {
  const int ct = a.Bs < 64 ? a.Bs : 64;
  const int cpb = ct < 4 ? ct : 4;
  const int tiles = (a.Bs + 63) / 64;
  hipLaunchKernelGGL(k_finalize, dim3(tiles * (ct / cpb)), dim3(kWG), 0, s, a);
}
void launch_zero(unsigned *p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(grid_flat(n)), dim3(kWG), 0, s, p, n);
}

}  // namespace pa
