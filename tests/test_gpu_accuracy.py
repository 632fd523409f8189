"""GPU: errors of the FP64 and FP32-refined paths against the FP64 oracle,
relative in the energy norm ||.||_W, printed per result: the exponential,
the averaged right-hand side, one averaged RK4 step and a 24-hour
integration, in the first workload's configuration (level 3, M = 8,
T = 1 h, 30-minute steps, ten seeded bumps).  Both GPU forms use the
Chebyshev mass solves (fused single-column steps, as in the benchmark)."""
import numpy as np
import pytest

from gpu_common import PARITY, block_max, bumps, onodes, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu

FORMS = {
    # FP64 steps, parity tolerances: the 1e-12 bar
    "fp64": (dict(**PARITY), 1e-12),
    # FP32 inner solves, FP64 refinement to 1e-12: the 1e-10 bar
    "fp32_refined": (dict(cheb_tol=1e-13, cg_rtol=1e-12, precision=1), 1e-10),
}


@pytest.mark.parametrize("form", list(FORMS))
def test_gpu_errors_against_oracle(form):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    kw, bar = FORMS[form]
    cfg = pa.solve_cfg(solver=pa.PA_SOLVER_CHEBYSHEV, backward=pa.PA_BACKWARD_CLENSHAW,
                       weight_cut=0.0, **kw)
    U = bumps(om, [0])
    avg = pa.Avg(8, 3600.0)
    err, emax = {}, {}
    ne = om.ne

    def note(key, got, ref):
        w, mx = rel_w(oo, got, ref), max(block_max(ne, got, ref))
        err[key], emax[key] = max(err.get(key, 0.0), w), max(emax.get(key, 0.0), mx)

    ts = [1800.0, -3600.0, 7200.0]
    out, _ = lo.expL_apply(ts, to_dev(mm.state(np.repeat(U, len(ts), axis=0))), cfg)
    got = mm.back(out.cpu().numpy())
    for j, t in enumerate(ts):
        note("exponential", got[j], oo.expL(lb, t, U[0], tol=1e-13, rtol=1e-14)[0])
    out, _ = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
    note("averaged RHS", mm.back(out.cpu().numpy())[0],
         oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14))
    Ud = to_dev(mm.state(U))
    ref = U[0].copy()
    for k in range(48):
        lo.step(avg, 1800.0, Ud, cfg)
        ref = oo.step(lb, *onodes(avg), 1800.0, ref, tol=1e-13, rtol=1e-14)
        if k == 0:
            note("one step", mm.back(Ud.cpu().numpy())[0], ref)
    note("24-hour state", mm.back(Ud.cpu().numpy())[0], ref)
    print(f"{form}: " + ", ".join(f"{k} {v:.2e} (max-norm {emax[k]:.2e})" for k, v in err.items()))
    for k in ("exponential", "averaged RHS", "one step"):
        assert err[k] < bar, (k, err[k])
        assert emax[k] < 10 * bar, (k, emax[k])
    # errors of the solves and of rounding add up over 48 steps
    assert err["24-hour state"] < 100 * bar
    assert emax["24-hour state"] < 1000 * bar
