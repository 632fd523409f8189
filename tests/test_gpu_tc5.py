"""GPU parity on the paper's own test case (Sec. 3: flow over an isolated
mountain, H = 5960 m, u0 = 20 m/s, g = 9.8 m/s^2): the bottom b != 0 enters
the depth flux -div(u (eta - b)) and the nonlinear energy.  The nonlinearity,
the averaged right-hand side (both backward forms), one averaged RK4 step of
900 s and the diagnostics against the oracle, at level 3, parity tolerances,
averaging window T = 1 h (M = 8: at least four nodes per period of the
fastest frequency, the paper's quadrature rule)."""
import functools

import numpy as np
import pytest

from gpu_common import PARITY, _ctx, check_parity, onodes, to_dev
from matching import MeshMap

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def tc5_pair(level):
    import oracle
    from paper_2103_07706_amd import inputs, pa
    ph = inputs.TC5_PHYSICS
    om = oracle.Mesh(level)
    lm = pa.Mesh(level)
    bo = inputs.williamson5_bottom(om.verts, om.cell_verts)
    bl = inputs.williamson5_bottom(lm.verts, lm.cell_verts)
    oo = oracle.Ops(om, g=ph.g, H=ph.H, Omega=ph.omega, b=bo)
    lo = pa.Ops(_ctx(), lm, g=ph.g, H=ph.H, omega=ph.omega, b=bl)
    lb = oracle.lambda_bar(oo, iters=200)
    lo.lambda_bar = lb
    U = inputs.williamson5_state(om.verts, om.cell_verts, om.edge_verts)
    return om, oo, lm, lo, MeshMap(om, lm), lb, U, bo


def test_tc5_bottom_maps_between_meshes():
    om, oo, lm, lo, mm, lb, U, bo = tc5_pair(3)
    from paper_2103_07706_amd import inputs
    bl = inputs.williamson5_bottom(lm.verts, lm.cell_verts)
    assert np.abs(bl - bo[mm.cell]).max() <= 1e-9 * bo.max() and bo.max() > 1000.0


def test_tc5_nonlinear_and_diagnostics():
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb, U, bo = tc5_pair(3)
    Ud = to_dev(mm.state(U)[None])
    out, _ = lo.swe_nonlinear(Ud, pa.solve_cfg(**PARITY))
    check_parity(oo, mm.back(out.cpu().numpy()[0]), oo.nonlinear(U, rtol=1e-14), 1e-12)
    d = lo.diagnostics(Ud)[0]
    ref = oo.diagnostics(U)
    for q, k in enumerate(["mass", "energy_linear", "energy_nonlinear", "hdiv_u", "l2_eta"]):
        assert abs(d[q] / ref[k] - 1) < 1e-13, (k, d[q], ref[k])


@pytest.mark.parametrize("backward", [0, 1])
def test_tc5_phase_avg_rhs_and_step(backward):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb, U, bo = tc5_pair(3)
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(backward=backward, weight_cut=0.0, **PARITY)
    out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)[None]), cfg)
    ref = oo.phase_avg_rhs(lb, *onodes(avg), U, tol=1e-13, rtol=1e-14)
    check_parity(oo, mm.back(out.cpu().numpy()[0]), ref, 1e-12, what=("nbar", backward))
    Ud = to_dev(mm.state(U)[None])
    lo.step(avg, 900.0, Ud, cfg)
    ref = oo.step(lb, *onodes(avg), 900.0, U, tol=1e-13, rtol=1e-14)
    check_parity(oo, mm.back(Ud.cpu().numpy()[0]), ref, 1e-12, what=("step", backward))
