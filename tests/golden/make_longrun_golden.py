"""Writes tests/golden/longrun_level5_m32_24h.txt: the oracle's state after a
24-hour integration of the averaged Lawson RK4 scheme (Sec. 2.3) at level 5
(20480 cells), M = 32 averaging terms over T = 2 h, dt = 1 h, 40 seeded
Gaussian bumps (member 0), at the throughput tolerances (Chebyshev
threshold 1e-6, mass solves to 1e-10).

Calls only the oracle (and the seeded input generator, which holds none of
the method's arithmetic).  Stored: the oracle's lambda_bar (the library is
given the same value), the diagnostics of the initial and final states, the
energy norm of the final state, and every 64th edge flux and cell depth of
the final state (oracle numbering, with the edge midpoint and the cell
centroid to 7 digits, so a reader can match any numbering by geometry).

Run from the repository root: python tests/golden/make_longrun_golden.py
(about ten minutes on one core).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2103_07706_amd import inputs  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "longrun_level5_m32_24h.txt")
LEVEL, M, T, DT, STEPS, NBUMPS, STRIDE = 5, 32, 7200.0, 3600.0, 24, 40, 64


def main():
    om = oracle.Mesh(LEVEL)
    oo = oracle.Ops(om)
    lb = oracle.lambda_bar(oo, iters=400)
    U = inputs.gaussian_bumps_state(om.verts, om.cell_verts, om.edge_verts, NBUMPS, 0)
    s, w = oracle.avg_nodes(M, T)
    d0 = oo.diagnostics(U)
    t0 = time.time()
    for k in range(STEPS):
        U = oo.step(lb, s, w, DT, U, tol=1e-6, rtol=1e-10)
        print(f"step {k + 1}/{STEPS} {time.time() - t0:.0f} s", flush=True)
    d1 = oo.diagnostics(U)
    mid = 0.5 * (om.verts[om.edge_verts[:, 0]] + om.verts[om.edge_verts[:, 1]])
    cen = om.verts[om.cell_verts].mean(axis=1)
    with open(OUT, "w") as f:
        f.write("# Oracle state after 24 hours of the averaged Lawson RK4 scheme (Sec. 2.3)\n")
        f.write(f"# level {LEVEL}, M {M}, T {T}, dt {DT}, {STEPS} steps, {NBUMPS} bumps seed 0,\n")
        f.write("# Chebyshev threshold 1e-6, mass solves 1e-10; written by make_longrun_golden.py\n")
        f.write(f"lambda_bar {float(lb)!r}\n")
        for key in ("mass", "energy_linear", "energy_nonlinear", "hdiv_u", "l2_eta"):
            f.write(f"initial_{key} {float(d0[key])!r}\n")
            f.write(f"final_{key} {float(d1[key])!r}\n")
        f.write(f"final_wnorm {float(oo.wnorm(U))!r}\n")
        f.write("# kind index x y z value (edge: midpoint, flux; cell: centroid, depth)\n")
        for e in range(0, om.ne, STRIDE):
            x = mid[e]
            f.write(f"e {e} {x[0]:.6e} {x[1]:.6e} {x[2]:.6e} {float(U[e])!r}\n")
        for c in range(0, om.nc, STRIDE):
            x = cen[c]
            f.write(f"c {c} {x[0]:.6e} {x[1]:.6e} {x[2]:.6e} {float(U[om.ne + c])!r}\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
