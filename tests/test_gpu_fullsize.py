"""GPU checks at the throughput workload's full size (level 6, 81920 cells,
122880 edges), in the configuration the benchmark times (M = 64, T = 2 h,
Chebyshev threshold 1e-6, mass solves to 1e-10, graph replay, Chebyshev
semi-iteration for the mass solves).

The oracle cannot evaluate all 64 terms here in reasonable time, so:
  * one averaging term at the largest phase shift (the longest
    exponentials) is compared with the oracle in parity mode;
  * the full 64-term result is checked through properties that hold at any
    size: zero mass of the depth tendency, agreement of the two independent
    backward formulations (per-term recurrences with fused weighted sum vs.
    one Clenshaw recurrence over term-combined right-hand sides), agreement
    of the two mass solvers, and invariance under graph replay.
"""
import numpy as np
import pytest

from gpu_common import PARITY, check_parity, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def l6():
    from paper_2103_07706_amd import inputs
    om, oo, lm, lo, mm, lb = pair(6, lambda_iters=120)
    U = inputs.gaussian_bumps_state(om.verts, om.cell_verts, om.edge_verts, 40, 0)
    return om, oo, lm, lo, mm, lb, U


def test_level6_single_term_matches_oracle(l6):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb, U = l6
    import oracle
    s = np.array([oracle.avg_nodes(64, 7200.0)[0][-1]])
    w = np.array([1.0])
    avg = pa.Avg(s=s, w=w)
    keep = pa.get_launch_tune()
    ref = oo.phase_avg_rhs(lb, s, w, U, tol=1e-13, rtol=1e-14)
    try:
        # CG; Chebyshev with six fused steps per launch (the benchmark's
        # autotuned shape at this level) and with one step per launch
        for solver, fs in ((0, 6), (1, 6), (1, 1)):
            pa.set_launch_tune(fused_steps=fs)
            cfg = pa.solve_cfg(solver=solver, weight_cut=0.0, **PARITY)
            out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)[None]), cfg)
            got = mm.back(out.cpu().numpy()[0])
            check_parity(oo, got, ref, 1e-12)
    finally:
        pa.set_launch_tune(**keep)


def test_level6_full_average_properties(l6):
    """In the launch shape the benchmark's autotuner picks at this level
    (six fused steps per launch, one row per thread for narrow blocks,
    FP32 solves on the 64-column block)."""
    import torch
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb, U = l6
    keep = pa.get_launch_tune()
    pa.set_launch_tune(fused_steps=6, narrow_rows_per_thread=1, wide_max_wg=2048, mixed_min_cols=64)
    try:
        _full_average(pa, torch, om, oo, lo, mm, U)
    finally:
        pa.set_launch_tune(**keep)


def _full_average(pa, torch, om, oo, lo, mm, U):
    avg = pa.Avg(64, 7200.0)
    Ud = to_dev(mm.state(U)[None])
    res = {}
    for name, bw, solver, graph, prec in [("clenshaw_cheb_graph", 1, 1, True, 0),
                                          ("clenshaw_cheb", 1, 1, False, 0),
                                          ("per_term_cheb", 0, 1, False, 0),
                                          ("clenshaw_cg", 1, 0, False, 0),
                                          ("clenshaw_fp32_refined", 1, 1, False, 1),
                                          ("per_term_fp32_refined", 0, 1, False, 1)]:
        cfg = pa.solve_cfg(backward=bw, solver=solver, cheb_tol=1e-6, cg_rtol=1e-10,
                           use_graph=graph, precision=prec)
        out = torch.empty_like(Ud)
        for _ in range(2 if graph else 1):
            _, st = lo.phase_avg_rhs(avg, Ud, cfg, out=out)
        res[name] = mm.back(out.cpu().numpy()[0])
        # every solve met its residual check: no Chebyshev or refined form
        # repeats the call (the refined forms' last inner round is sized to
        # what remains); a CG form may repeat once with polling when the
        # context's iteration budget, learned on other problems, was short
        assert st["fallbacks"] <= (1 if solver == 0 else 0), (name, st)
        if solver == 1:  # Chebyshev solves check and report their true residuals
            assert 0 < st["resid_max"] <= 1e-10, (name, st["resid_max"])
        if prec:
            assert st["refinements"] > 0, name
    ref = res["clenshaw_cheb"]
    area = oo.export()["area"]
    for name, v in res.items():
        # mass of the depth tendency vanishes
        assert abs(np.sum(area * v[om.ne:])) <= 1e-12 * np.sum(np.abs(area * v[om.ne:])), name
        # the formulations agree to the solve tolerance
        assert rel_w(oo, v, ref) < 1e-8, (name, rel_w(oo, v, ref))
    assert np.array_equal(res["clenshaw_cheb_graph"], ref)
