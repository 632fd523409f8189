// Device scratch for the allocation-free entry point (pa_phase_avg_rhs_noalloc
// in include/pa.h): a file-scope device array stands in for the caller's
// workspace.  Each GPU the library runs on holds its own copy for the life of
// the process; its device address is looked up once per device with that
// device current, and only that address is handed to kernels and copies (the
// array's name in host code is a host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "pa_engine.h"

namespace {
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The device address of this device's scratch array (looked up on the first
// call for the device, with the device current).
void *scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) throw pa::Error(PA_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    PA_HIP(hipSetDevice(device));
    void *p = nullptr;
    PA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw pa::Error(PA_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

}  // namespace

extern "C" int pa_phase_avg_rhs_noalloc(pa_ctx *ctx, const pa_ops *ops, const pa_avg *avg,
                                        int members, const double *U_dev, double *Nbar_dev,
                                        const pa_solve_cfg *cfg, pa_stats *stats) {
  return pa::guard([&] {
    if (!ctx || !ops || !avg || !U_dev || !Nbar_dev || members < 1)
      throw pa::Error(PA_EINVAL, "bad arguments");
    if (!ops->dev) throw pa::Error(PA_EINVAL, "operators not bound (pa_ops_bind)");
    pa_solve_cfg c;
    pa_solve_cfg_default(&c);
    if (cfg) c = *cfg;
    c.use_graph = 0;  // instantiating a graph allocates device memory
    // the call's workspace and that of its FP64 CG repeat must fit
    pa_solve_cfg cg = c;
    cg.solver = PA_SOLVER_CG;
    cg.precision = PA_FP64;
    const size_t need =
        std::max(pa::workspace_bytes(ops, avg, members, c), pa::workspace_bytes(ops, avg, members, cg));
    if (need > kScratchBytes)
      throw pa::Error(PA_ENOMEM, "the problem needs " + std::to_string((need + (1 << 20) - 1) >> 20) +
                                     " MiB of workspace; the static scratch holds " +
                                     std::to_string(kScratchBytes >> 20) + " MiB");
    void *ws = scratch_address(ctx->device);
    pa::phase_avg_rhs_call(ctx, ops, avg, members, U_dev, Nbar_dev, ws, kScratchBytes, c, stats);
  });
}
