// Internal declarations of libpa (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstring>
#include <map>
#include <new>
#include <cstdint>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pa.h"

namespace pa {

// Error carried to the C ABI boundary, where it becomes a status code.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Ritz bounds of the symmetric operator y = S(x) of size n (Lanczos, fixed
// start vector, 'steps' steps).
void ritz_bounds(int n, const std::function<void(const std::vector<double> &, std::vector<double> &)> &S,
                 int steps, double *lmin, double *lmax);

// Thread-local message returned by pa_last_error.
std::string &last_error();

// Runs f, turning any exception into a status code and the error message.
template <class F>
int guard(F &&f) {
  try {
    f();
    return PA_OK;
  } catch (const Error &e) {
    last_error() = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    last_error() = "host out of memory";
    return PA_ENOMEM;
  } catch (const std::exception &e) {
    last_error() = e.what();
    return PA_EINVAL;
  } catch (...) {
    last_error() = "unknown error";
    return PA_EINVAL;
  }
}

#define PA_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::pa::Error(PA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Waits for the stream.  A launch that failed to start (launch
// configuration, missing code object) leaves its error for hipGetLastError
// only, so that is checked first.
inline void sync_checked(hipStream_t s) {
  PA_HIP(hipGetLastError());
  PA_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- host mesh
struct Mesh {
  int level = 0;
  double radius = 0;
  std::vector<double> xyz;      // nv*3
  std::vector<int32_t> tri;     // nc*3, CCW from outside
  std::vector<int32_t> cedge;   // nc*3, edge opposite local vertex i
  std::vector<int32_t> csgn;    // nc*3, +1 if the edge normal leaves the cell
  std::vector<int32_t> ecell;   // ne*2, (c0, c1), c0 < c1
  std::vector<int32_t> evert;   // ne*2, a -> b counter-clockwise about c0
  int nv() const { return (int)xyz.size() / 3; }
  int nc() const { return (int)tri.size() / 3; }
  int ne() const { return (int)ecell.size() / 2; }
};
Mesh build_icosahedral(int level, double radius);

// Number of doubles of per-cell geometry used by the nonlinear kernels:
// vertices p[3][3], unit normal k[3], area, grad of barycentrics gl[3][3],
// side lengths len[3]; padded to 32 (256 bytes).
constexpr int kCellGeo = 32;
// Per-edge tangential-trace table: tau[side][gauss][j] (2*2*3).
constexpr int kEdgeTau = 12;
// Per cell: the nonlinear cell term as forms in the cell's edge fluxes U
// (three symmetric 3x3 forms, then the facet coefficients of the two Gauss
// points of each side; built by nl_cell_forms with the operators)
constexpr int kNlForm = 72;
// Row parts of the fused-step mass-solve kernel: part p holds the kPartRows
// edges [p kPartRows, (p + 1) kPartRows).  Ring 1 of a part is the set of
// other edges its rows' ELL columns reach, ring r + 1 the edges ring r's
// columns reach outside the part and rings 1..r.  kFusedMax - 1 rings are
// kept, at most kHaloMax rows in all per part (fewer rings on a mesh where
// they do not fit).
constexpr int kPartRows = 512;  // also the kernel's workgroup size: one row a thread
constexpr int kHaloMax = 1024;
constexpr int kFusedMax = 6;

// Device-resident operator arrays (pointers into the caller's buffer).
struct DevOps {
  int ne = 0, nc = 0;
  double g = 0, H = 0;
  const int32_t *ell_col = nullptr;   // ne*5: self, two of c0, two of c1
  const double *mass = nullptr;       // ne*5
  const double *cor = nullptr;        // ne*5
  const double *graddiv = nullptr;    // ne*5: D' A^-1 D on the same pattern
  const float *mass32 = nullptr;      // ne*5
  const double *dinv = nullptr;       // ne
  const float *dinv32 = nullptr;      // ne
  const int32_t *ecell = nullptr;     // ne*2
  const int32_t *cidx = nullptr;      // ne*2: 3*c + local index in c0, c1
  const int32_t *cell_edges = nullptr;// nc*12: the cell's edges, then per local edge a the
                                      // edges of the cell across a (48-byte records)
  const double *tau = nullptr;        // ne*12
  const int32_t *cedge = nullptr;     // nc*3
  const int32_t *csgn = nullptr;      // nc*3
  const int32_t *cnbr = nullptr;      // nc*3: cell across local edge a
  const double *area = nullptr;       // nc
  const double *inv_area = nullptr;   // nc
  const double *bottom = nullptr;     // nc
  const double *cgeo = nullptr;       // nc*kCellGeo
  const double *nlform = nullptr;     // nc*kNlForm
  // row parts (see kPartRows): hparts parts, rings 1..fused_max-1 kept
  int hparts = 0, fused_max = 1;
  const int32_t *ring_cnt = nullptr;  // hparts*8: rows of rings 1..r of part p, r = 1..kFusedMax-1
  const int32_t *ring_row = nullptr;  // hparts*kHaloMax: part p's ring rows from p*kHaloMax,
                                      // ring by ring, ascending within a ring, then -1
  const uint16_t *hloc = nullptr;     // 5*ne, [slot][row]: ELL column as a part-local index
                                      // (row offset in the part, or kPartRows + ring position)
  const uint16_t *ring_loc = nullptr; // hparts*kHaloMax*5: the same for the ring rows
                                      // (rings 1..fused_max-2; others 0)
};

// Learned preconditioner on the device: P = G G^T and P M as column-major
// ELL tables ([slot][row], padding col = row, value 0) of packed entries
// (x = column, y = FP32 value bits), one 8-byte load per entry.
struct DevLp {
  int wp = 0, wpm = 0;
  const uint2 *p = nullptr;
  const uint2 *pm = nullptr;
};

// Launch shape of the row-parallel kernels (set by the autotuner).
struct LaunchTune {
  int narrow_rows_per_thread = 4;  // batches of <= 4 columns
  int wide_max_wg = 2048;          // workgroups per column tile, wider batches
  int lp_min_cols = 8;             // learned mass-solve steps on blocks this wide or wider
  int mixed_min_cols = 8;          // FP32-refined mass solves on blocks this wide or wider
  int fused_steps = 6;             // single-column Jacobi Chebyshev solves: steps per launch (1 to kFusedMax)
  bool operator==(const LaunchTune &o) const {
    return narrow_rows_per_thread == o.narrow_rows_per_thread && wide_max_wg == o.wide_max_wg &&
           lp_min_cols == o.lp_min_cols && mixed_min_cols == o.mixed_min_cols &&
           fused_steps == o.fused_steps;
  }
};

// What a captured averaged-RHS graph depends on.
// Field-wise equality of solve configurations (no padding compared).
inline bool same_cfg(const pa_solve_cfg &a, const pa_solve_cfg &b) {
  return a.precision == b.precision && a.backward == b.backward && a.maxit == b.maxit &&
         a.growth_guard == b.growth_guard && a.cg_rtol == b.cg_rtol && a.cheb_tol == b.cheb_tol &&
         a.weight_cut == b.weight_cut && a.inner_rtol == b.inner_rtol && a.use_graph == b.use_graph &&
         a.solver == b.solver && a.precond == b.precond && a.exponential == b.exponential &&
         a.rexi_nodes == b.rexi_nodes && a.rexi_eta0 == b.rexi_eta0;
}

// Objects whose contents a captured graph bakes in (operators and their
// bound buffers, averaging nodes) carry a generation number, unique over
// the process and renewed whenever the contents or the device buffers
// change: a new object at a freed object's address never matches a key.
uint64_t next_generation();

struct GraphKey {
  const void *in = nullptr, *out = nullptr, *ws = nullptr;
  uint64_t ops_gen = 0, avg_gen = 0;
  int members = 0, budget = 0;
  double lambda_bar = 0;
  pa_solve_cfg cfg{};
  LaunchTune tune{};
  bool operator==(const GraphKey &o) const {
    return ops_gen == o.ops_gen && avg_gen == o.avg_gen && in == o.in && out == o.out &&
           ws == o.ws && members == o.members && budget == o.budget &&
           lambda_bar == o.lambda_bar && tune == o.tune && same_cfg(cfg, o.cfg);
  }
};

// Launch shape in force for the kernels the calling thread enqueues: set by
// each call for its duration (TuneScope) from the operators' own shape, a
// batch item's shape or the process default.
LaunchTune launch_default();
void set_launch_default(const LaunchTune &t);
LaunchTune clamp_tune(LaunchTune t);
struct TuneScope {
  explicit TuneScope(const LaunchTune &t);
  ~TuneScope();
  TuneScope(const TuneScope &) = delete;
  TuneScope &operator=(const TuneScope &) = delete;

 private:
  const LaunchTune *prev_;
};

}  // namespace pa

// ----------------------------------------------------------- opaque handles
struct pa_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void *host_flag = nullptr;  // pinned host word for convergence polling
  // learned CG iterations per solve, per tolerance (absent: poll)
  std::map<double, int> cg_budget;
  // iterations of the last rational-exponential solve (first poll point)
  int rexi_pred = 0;
  // graph replay of the averaged right-hand side
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  pa::GraphKey graph_key{};
  pa_stats graph_stats{};
  // measurement hook (pa_ctx_profile)
  int prof_kernel = 0;
  std::vector<hipEvent_t> prof_pool;
  int64_t prof_launches = 0, prof_work = 0;
  double prof_ms = 0.0, prof_bytes = 0.0, prof_units = 0.0;
};

struct pa_mesh {
  pa::Mesh m;
};

struct pa_ops {
  const pa_mesh *mesh = nullptr;
  uint64_t gen = 0;  // renewed at creation, bind, learned-table attach and bind
  // the operators' own launch shape (pa_ops_set_tune, pa_autotune); without
  // one, calls take the process default
  mutable pa::LaunchTune tune{};
  mutable bool has_tune = false;
  pa::LaunchTune effective_tune() const { return has_tune ? tune : pa::launch_default(); }
  int ne = 0, nc = 0;
  double g = 0, H = 0, omega = 0, lambda_bar = 0;
  double mass_eig_min = 0, mass_eig_max = 0;  // Ritz bounds of D^-1 M
  // host copies, in upload order
  std::vector<int32_t> ell_col, ecell, cidx, cell_edges, cedge, csgn, cnbr;
  std::vector<double> mass, cor, graddiv, dinv, area, inv_area, bottom, cgeo, nlform, tau;
  std::vector<float> mass32, dinv32;
  int hparts = 0, fused_max = 1;
  int fused_cpp = 0;  // cells per part in a set-up launch (0: no set-up launches)
  int fused_slots[pa::kFusedMax + 1][pa::kFusedMax] = {};  // per S and step: ring slots
                                                           // (see ChebFusedArgs)
  std::vector<int32_t> ring_cnt, ring_row;
  std::vector<uint16_t> hloc, ring_loc;
  size_t dev_bytes = 0;
  void *dev = nullptr;
  pa::DevOps d;
  // learned preconditioner (pa_ops_lp_attach / pa_ops_lp_bind)
  int lp_wp = 0, lp_wpm = 0;
  std::vector<int32_t> lp_pcol, lp_pmcol;
  std::vector<float> lp_pval, lp_pmval;
  double lp_eig_min = 0, lp_eig_max = 0;
  bool lp_ready = false;   // tables built
  void *lp_dev = nullptr;  // bound device copy
  pa::DevLp lp;
};

struct pa_avg {
  uint64_t gen = pa::next_generation();  // nodes and weights never change
  std::vector<double> s, w;
};
