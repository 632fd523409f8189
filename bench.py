"""Throughput of the phase-averaged right-hand side on one MI355X.

One step = one evaluation of Nbar(U) = sum_m w_m exp(-s_m L) N(exp(s_m L) U)
on the level-6 icosahedral mesh (81920 cells, 122880 edges) with M = 64
averaging terms over T = 2 h, FP64, Chebyshev threshold 1e-6 and every mass
solve to a relative residual of 1e-10 (the throughput workload), with the
input state already resident in device memory.  Prints one JSON line.

Also reported: the roofline position of the dominant kernel (HIP events
around each of its launches during the timed region, algorithmic bytes from
the library's count of active columns), and the oracle timed on a bounded
sample of the same workload on the host cores (cpu_baseline).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="l6_m64")
    ap.add_argument("--backward", default="clenshaw", choices=["per_term", "clenshaw"])
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--solver", default="chebyshev", choices=["cg", "chebyshev"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_refined"])
    ap.add_argument("--autotune", type=int, default=1)
    ap.add_argument("--cpu-baseline", dest="cpu", type=int, default=1)
    ap.add_argument("--cpu-terms", type=int, default=4)
    return ap.parse_args()


def kernel_source_hash():
    src = os.path.join(ROOT, "paper_2103_07706_amd", "csrc", "pa_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_from_profiles(kernel, workload, backward):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{backward}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(wl, lam, nterms):
    """The oracle (single-threaded C, FP64) on a sample of the workload's
    averaging terms: every (M / nterms)-th term, scaled to a whole Nbar."""
    import numpy as np

    import oracle
    from paper_2103_07706_amd import inputs
    om = oracle.Mesh(wl.level)
    oo = oracle.Ops(om, g=wl.phys.g, H=wl.phys.H, Omega=wl.phys.omega)
    U = inputs.gaussian_bumps_state(om.verts, om.cell_verts, om.edge_verts, wl.nbumps, 0,
                                    wl.phys)
    s, w = oracle.avg_nodes(wl.M, wl.T)
    idx = list(range(wl.M // (2 * nterms), wl.M, max(1, wl.M // nterms)))[:nterms]
    t0 = time.perf_counter()
    oo.phase_avg_rhs(lam, s[idx], w[idx], U, tol=1e-6, rtol=1e-10)
    dt = time.perf_counter() - t0
    per_eval = dt * wl.M / len(idx)
    return {"value": 1.0 / per_eval, "unit": "Nbar/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(idx)} of {wl.M} averaging terms (indices {idx}) of one Nbar at "
                      f"level {wl.level}, scaled by {wl.M}/{len(idx)}; {dt:.1f} s measured"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards over averaging terms or members, see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2103_07706_amd import inputs, pa
    wl = inputs.WORKLOADS[args.workload]
    ctx = pa.Context(0)
    mesh = pa.Mesh(wl.level)
    ops = pa.Ops(ctx, mesh, g=wl.phys.g, H=wl.phys.H, omega=wl.phys.omega)
    lam = ops.estimate_lambda(iters=200, safety=1.05)
    import numpy as np
    U = torch.tensor(
        np.stack([inputs.gaussian_bumps_state(mesh.verts, mesh.cell_verts, mesh.edge_verts,
                                              wl.nbumps, m, wl.phys) for m in range(wl.members)]),
        dtype=torch.float64, device="cuda:0")
    avg = pa.Avg(wl.M, wl.T)
    bw = pa.PA_BACKWARD_PER_TERM if args.backward == "per_term" else pa.PA_BACKWARD_CLENSHAW
    solver = pa.PA_SOLVER_CG if args.solver == "cg" else pa.PA_SOLVER_CHEBYSHEV
    prec = pa.PA_FP64 if args.precision == "fp64" else pa.PA_FP32_REFINED
    cfg = pa.solve_cfg(backward=bw, cheb_tol=1e-6, cg_rtol=1e-10, use_graph=bool(args.graph),
                       solver=solver, precision=prec)
    out = torch.empty_like(U)
    tune = None
    if args.autotune:
        tune = ops.autotune(avg, U, cfg)
        print(f"autotune {tune}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ops.phase_avg_rhs(avg, U, cfg, out=out)
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for i in range(args.steps):
        _, stats = ops.phase_avg_rhs(avg, U, cfg, out=out)
        print(f"step {i} {stats['device_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    # the dominant kernel, timed with HIP events around each of its launches
    # over the same number of steps (events add small gaps between kernels,
    # so this pass is kept apart from the throughput measurement)
    kernel = "k_cheb_iter" if args.solver == "chebyshev" else "k_cg_iter"
    ctx.profile(pa.PA_KERNEL_CHEB_ITER if args.solver == "chebyshev" else pa.PA_KERNEL_CG_ITER)
    for i in range(args.steps):
        ops.phase_avg_rhs(avg, U, cfg, out=out)
    prof = ctx.profile_read()
    ctx.profile(pa.PA_KERNEL_NONE)
    value = wl.members * args.steps / elapsed
    avg_ms = prof["total_ms"] / max(1, prof["launches"])
    achieved = prof["bytes"] / (prof["total_ms"] * 1e-3) / 1e9 if prof["total_ms"] > 0 else 0.0
    traffic = traffic_from_profiles(kernel, args.workload, args.backward)
    rec = {
        "metric": "phase-avg RHS evals/s (L6 mesh, M=64)",
        "value": value,
        "unit": "Nbar/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "level": wl.level, "cells": mesh.nc,
                   "edges": mesh.ne, "M": wl.M, "T_s": wl.T, "members": wl.members,
                   "cheb_tol": 1e-6, "cg_rtol": 1e-10, "backward": args.backward,
                   "precision": args.precision, "preconditioner": "jacobi", "lambda_bar": lam,
                   "mass_solver": args.solver,
                   "kmax": stats["kmax"], "ksum": stats["ksum"], "terms": stats["terms"],
                   "cg_iters_max": stats["cg_iters_max"], "solves": stats["solves"],
                   "graph": bool(stats["graph"]), "cg_budget": stats["budget"],
                   "launch_tune": tune},
        "roofline": {"bound": "hbm", "kernel": kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": 1e3 * avg_ms,
                     "launches": prof["launches"],
                     "algorithmic_bytes_per_launch": prof["bytes"] / max(1, prof["launches"])},
    }
    if args.cpu:
        print("cpu baseline ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(wl, lam, args.cpu_terms)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
