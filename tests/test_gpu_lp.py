"""GPU: the learned mass-matrix preconditioner.  Network outputs and loss
gradients of the HIP kernels against the FP64 reference (oracle/lp_ref.py)
on the same parameters and probes (mapped between the two mesh numberings);
training on the GPU; solves with the learned preconditioner against the
oracle and against the Jacobi-preconditioned path."""
import functools

import numpy as np
import pytest

from gpu_common import PARITY, bumps, check_parity, onodes, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _graph(level):
    from oracle import lp_ref
    om, oo, lm, lo, mm, lb = pair(level)
    return lp_ref.Graph(om, oo)


def _theta(seed, scale=0.3):
    """Parameters exactly representable in FP32, shared by both sides."""
    from oracle import lp_ref
    rng = np.random.default_rng(seed)
    th = lp_ref.init_params(seed) + scale * rng.standard_normal(lp_ref.n_params())
    return th.astype(np.float32)


def _lib_pairs(lm):
    """Library pair columns: for edge i the other two edges of its first
    cell, then of its second cell, in the cells' edge order."""
    pj = np.zeros((lm.ne, 4), np.int64)
    for i in range(lm.ne):
        k = 0
        for c in lm.edge_cells[i]:
            for e in lm.cell_edges[c]:
                if e != i:
                    pj[i, k] = e
                    k += 1
    return pj


@pytest.mark.parametrize("bf16", [False, True])
def test_gpu_lp_ghat_matches_oracle(bf16):
    from oracle import lp_ref
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(2)
    g = _graph(2)
    th = _theta(3)
    lp = pa.LearnedPrecond()
    lp.params = th
    gd, go = lp.ghat(lo, bf16=bf16)
    _, gd_ref, _, goff_ref = lp_ref.forward(th.astype(np.float64), g)
    tol = 3e-2 if bf16 else 1e-5
    e = mm.edge
    assert np.abs(gd - gd_ref[e]).max() <= tol * np.abs(gd_ref).max()
    ref_pair = {(int(i), int(j)): v for i, j, v in zip(g.pi, g.pj, goff_ref)}
    pj = _lib_pairs(lm)
    want = np.array([[ref_pair[(int(e[i]), int(e[pj[i, s]]))] * mm.sign[i] * mm.sign[pj[i, s]]
                      for s in range(4)] for i in range(lm.ne)])
    assert np.abs(go - want).max() <= tol * np.abs(want).max()


@pytest.mark.parametrize("bf16", [False, True])
def test_gpu_lp_gradient_matches_oracle(bf16):
    """Loss and full parameter gradient: FP32 matrix-core layers within
    1e-6 of the FP64 reference, BF16 within 1e-2 (relative, whole vector).
    Parameters: the initial network plus N(0, 0.1^2) noise on every entry,
    so that both heads and every layer carry gradient (the initial heads are
    zero); larger noise drives the loss orders of magnitude above any
    trained or initial value and BF16 rounding of the activations grows
    with it."""
    from oracle import lp_ref
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(2)
    g = _graph(2)
    th = _theta(4, scale=0.1)
    rng = np.random.default_rng(8)
    Z = rng.choice([-1.0, 1.0], size=(om.ne, 4))
    Zl = Z[mm.edge] * mm.sign[:, None]
    lp = pa.LearnedPrecond()
    lp.params = th
    L, grad = lp.loss_grad(lo, Zl, bf16=bf16)
    L_ref, grad_ref = lp_ref.loss_grad(th.astype(np.float64), g, Z)
    tol = 1e-2 if bf16 else 1e-6
    assert abs(L - L_ref) <= tol * L_ref, (L, L_ref)
    err = np.linalg.norm(grad - grad_ref) / np.linalg.norm(grad_ref)
    print(f"bf16={bf16}: loss {L:.6e} vs {L_ref:.6e}, gradient relative error {err:.2e}")
    assert err <= tol


@functools.lru_cache(maxsize=None)
def _trained():
    from paper_2103_07706_amd import pa
    lp = pa.LearnedPrecond(seed=5)
    ops = [pair(2)[3], pair(3)[3]]
    st = lp.train(ops, steps=200, probes=8, lr=3e-3, bf16=True, seed=11)
    return lp, st


def test_gpu_lp_training_lowers_loss():
    lp, st = _trained()
    print(st)
    assert st["steps"] == 200
    assert st["loss_last"] < 0.2 * st["loss_first"]


def _steps(lo_, hi_, rtol):
    a, b = 0.95 * lo_, 1.02 * hi_
    return int(np.ceil(np.arccosh(2 / rtol) / np.arccosh((a + b) / (b - a)))) + 2


def test_gpu_lp_attach_narrows_the_spectrum():
    """Applied to a finer mesh than it was trained on, the learned P M has a
    tighter spectrum than Jacobi, so the Chebyshev solves take fewer steps."""
    from paper_2103_07706_amd import pa
    lp, _ = _trained()
    lo = pair(4)[3]
    info = pa.attach_learned(lo, lp, bf16=True)
    print(info)
    kl = _steps(info["eig_min"], info["eig_max"], 1e-10)
    kj = _steps(info["jacobi_eig_min"], info["jacobi_eig_max"], 1e-10)
    assert info["eig_min"] > 0
    assert kl < kj, (kl, kj)


def _set_lp_min_cols(pa, n):
    t = pa.LaunchTune()
    pa._check(pa.lib().pa_get_launch_tune(t))
    keep = t.lp_min_cols
    t.lp_min_cols = n
    pa._check(pa.lib().pa_set_launch_tune(t))
    return keep


@pytest.mark.parametrize("lp_min_cols", [1, 8])
def test_gpu_lp_solves_parity(lp_min_cols):
    """Averaged right-hand side with the learned preconditioner in the
    Chebyshev mass solves: parity with the oracle (Jacobi CG) at 1e-12, same
    result as the Jacobi Chebyshev path to the solve tolerance, fewer steps
    in the learned solves, graph replays equal to eager.  lp_min_cols = 1:
    every solve learned (single-column recurrences take the one-kernel step);
    8: only the 16-column nonlinear solves (two-kernel step)."""
    import torch
    from paper_2103_07706_amd import pa
    lp, _ = _trained()
    om, oo, lm, lo, mm, lb = pair(3)
    pa.attach_learned(lo, lp, bf16=True)
    keep = _set_lp_min_cols(pa, lp_min_cols)
    try:
        U = bumps(om, [2])
        Ud = to_dev(mm.state(U))
        avg = pa.Avg(16, 3600.0)
        base = dict(backward=pa.PA_BACKWARD_CLENSHAW, solver=pa.PA_SOLVER_CHEBYSHEV)
        out_l, st_l = lo.phase_avg_rhs(avg, Ud, pa.solve_cfg(
            precond=pa.PA_PRECOND_LEARNED, weight_cut=0.0, **base, **PARITY))
        out_j, st_j = lo.phase_avg_rhs(avg, Ud, pa.solve_cfg(weight_cut=0.0, **base, **PARITY))
        assert st_l["precond"] == pa.PA_PRECOND_LEARNED and st_j["precond"] == pa.PA_PRECOND_JACOBI
        if lp_min_cols == 1:
            assert st_l["lp_solves"] == st_l["solves"]
        else:
            assert 1 <= st_l["lp_solves"] < st_l["solves"]
        assert st_j["lp_solves"] == 0
        assert st_l["cg_iters"] < st_j["cg_iters"]  # fewer steps in total
        ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
        got = mm.back(out_l.cpu().numpy())[0]
        check_parity(oo, got, ref, 1e-12)
        gj = mm.back(out_j.cpu().numpy())[0]
        assert rel_w(oo, got, gj) < 1e-12
        # metric tolerances, graph capture and replay
        mcfg = dict(precond=pa.PA_PRECOND_LEARNED, cheb_tol=1e-6, cg_rtol=1e-10, **base)
        eager, _ = lo.phase_avg_rhs(avg, Ud, pa.solve_cfg(use_graph=False, **mcfg))
        eager = eager.cpu().numpy()
        gcfg = pa.solve_cfg(use_graph=True, **mcfg)
        out = torch.empty_like(Ud)
        for i in range(3):
            out.fill_(float("nan"))
            _, st = lo.phase_avg_rhs(avg, Ud, gcfg, out=out)
            assert st["graph"] == 1 and st["precond"] == pa.PA_PRECOND_LEARNED
            assert np.array_equal(out.cpu().numpy(), eager), i
            lo.swe_nonlinear(Ud)
            torch.cuda.synchronize()
    finally:
        _set_lp_min_cols(pa, keep)


def test_gpu_lp_requires_binding():
    from paper_2103_07706_amd import pa
    from gpu_common import _ctx
    lm = pa.Mesh(2)
    lo = pa.Ops(_ctx(), lm)
    lo.lambda_bar = pair(2)[5]
    U = to_dev(np.zeros((1, lo.n)))
    cfg = pa.solve_cfg(precond=pa.PA_PRECOND_LEARNED, solver=pa.PA_SOLVER_CHEBYSHEV)
    with pytest.raises(pa.PAError) as ei:
        lo.phase_avg_rhs(pa.Avg(4, 1000.0), U, cfg)
    assert ei.value.code == pa.PA_EINVAL
