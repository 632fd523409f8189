"""GPU checks at the largest configured size (level 7: 327680 cells, 491520
edges), where the learned preconditioner trained on levels 4-6 is applied.

One averaging term at the largest phase shift of the M = 64, T = 2 h
average (the longest exponentials) is compared with the oracle in parity
mode, through the Jacobi Chebyshev path (six fused steps per launch, the
benchmark's shape) and through the learned preconditioner in every mass
solve; the learned solves must also take fewer Chebyshev steps.  lambda_bar
comes from the oracle's Lanczos estimate (60 steps: about 20 s on one core
at this size; the oracle term takes about 40 s).
"""
import numpy as np
import pytest

from gpu_common import PARITY, _ctx, check_parity, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def l7():
    from paper_2103_07706_amd import inputs, pa
    om, oo, lm, lo, mm, lb = pair(7, lambda_iters=60)
    U = inputs.gaussian_bumps_state(om.verts, om.cell_verts, om.edge_verts, 40, 0)
    import oracle
    s = np.array([oracle.avg_nodes(64, 7200.0)[0][-1]])
    w = np.array([1.0])
    print(f"level 7: oracle term at s = {s[0]} s", flush=True)
    ref = oo.phase_avg_rhs(lb, s, w, U, tol=1e-13, rtol=1e-14)
    return om, oo, lm, lo, mm, lb, U, s, w, ref


def test_level7_single_term_jacobi_and_learned(l7):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb, U, s, w, ref = l7
    avg = pa.Avg(s=s, w=w)
    Ud = to_dev(mm.state(U)[None])
    keep = pa.get_launch_tune()
    try:
        pa.set_launch_tune(fused_steps=6)
        base = dict(solver=pa.PA_SOLVER_CHEBYSHEV, weight_cut=0.0, **PARITY)
        out_j, st_j = lo.phase_avg_rhs(avg, Ud, pa.solve_cfg(**base))
        got_j = mm.back(out_j.cpu().numpy()[0])
        check_parity(oo, got_j, ref, 1e-12)
        # the learned preconditioner, trained on levels 4-6 only
        lp = pa.LearnedPrecond(seed=5)
        train_ops = [pa.Ops(_ctx(), pa.Mesh(level)) for level in (4, 5, 6)]
        tr = lp.train(train_ops, steps=100, probes=8, lr=3e-3, bf16=True, seed=11)
        assert tr["loss_last"] < tr["loss_first"]
        pa.attach_learned(lo, lp, bf16=True)
        pa.set_launch_tune(lp_min_cols=1)
        out_l, st_l = lo.phase_avg_rhs(avg, Ud, pa.solve_cfg(precond=pa.PA_PRECOND_LEARNED, **base))
        assert st_l["precond"] == pa.PA_PRECOND_LEARNED
        assert st_l["lp_solves"] == st_l["solves"] and st_l["fallbacks"] == 0
        assert st_l["cg_iters"] < st_j["cg_iters"], (st_l["cg_iters"], st_j["cg_iters"])
        got_l = mm.back(out_l.cpu().numpy()[0])
        check_parity(oo, got_l, ref, 1e-12)
    finally:
        pa.set_launch_tune(**keep)
