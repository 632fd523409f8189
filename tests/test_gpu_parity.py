"""GPU parity: the HIP path through the C ABI against the oracle, element by
element after mapping the two mesh numberings, on the same seeded inputs.

Tolerance: relative 1e-12 in the energy norm ||.||_W (where L is skew and
the exponential is an isometry) for FP64 with both sides in parity mode
(Chebyshev threshold 1e-13, CG to 1e-14), plus a max-norm check per block.
"""
import numpy as np
import pytest

from gpu_common import PARITY, bumps, check_parity, onodes, pair, rel_w, to_dev

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _maxrel(a, b, ne):
    ua, ub = a[..., :ne], b[..., :ne]
    ea, eb = a[..., ne:], b[..., ne:]
    return max(np.abs(ua - ub).max() / np.abs(ub).max(), np.abs(ea - eb).max() / np.abs(eb).max())


@pytest.mark.parametrize("level", [2, 3])
def test_gpu_expL_parity(level):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(level)
    ts = [600.0, -1800.0, 3600.0, 0.0, 7200.0]
    U = bumps(om, range(len(ts)))
    out, st = lo.expL_apply(ts, to_dev(mm.state(U)), pa.solve_cfg(**PARITY))
    got = mm.back(out.cpu().numpy())
    for j, t in enumerate(ts):
        ref, K = oo.expL(lb, t, U[j], tol=1e-13, rtol=1e-14)
        check_parity(oo, got[j], ref, TOL)
    assert st["cg_iters_max"] <= 30


def test_gpu_nonlinear_parity():
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0, 1, 2])
    out, st = lo.swe_nonlinear(to_dev(mm.state(U)), pa.solve_cfg(**PARITY))
    got = mm.back(out.cpu().numpy())
    for j in range(3):
        ref = oo.nonlinear(U[j], rtol=1e-14)
        check_parity(oo, got[j], ref, TOL)
        assert _maxrel(got[j], ref, om.ne) < 1e-11


@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("backward", ["per_term", "clenshaw"])
@pytest.mark.parametrize("M,T", [(8, 3600.0), (5, 2000.0), (1, 1000.0)])
def test_gpu_phase_avg_rhs_parity(backward, M, T, solver):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0])
    avg = pa.Avg(M, T)
    bw = pa.PA_BACKWARD_PER_TERM if backward == "per_term" else pa.PA_BACKWARD_CLENSHAW
    cfg = pa.solve_cfg(backward=bw, solver=solver, weight_cut=0.0, **PARITY)
    out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
    got = mm.back(out.cpu().numpy())[0]
    ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
    check_parity(oo, got, ref, TOL)
    assert st["terms"] == M


def test_gpu_phase_avg_members_independent():
    """Several ensemble members in one call equal separate calls."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = mm.state(bumps(om, [3, 4, 5]))
    avg = pa.Avg(6, 3000.0)
    cfg = pa.solve_cfg(**PARITY)
    allm, _ = lo.phase_avg_rhs(avg, to_dev(U), cfg)
    allm = allm.cpu().numpy()
    for j in range(3):
        one, _ = lo.phase_avg_rhs(avg, to_dev(U[j:j + 1]), cfg)
        ref = mm.back(one.cpu().numpy()[0])
        assert rel_w(oo, mm.back(allm[j]), ref) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_gpu_wide_ensemble_parity(precision):
    """64 members in one call (level 3, M = 8): the recurrences run on
    64-column blocks and the solve of N on a 512-column block, so the block
    kernels take their one-row-a-wave form (row tables read through the
    scalar unit), including the FP32 step over four columns a lane at 256 or
    more columns.  Sampled members against the FP64 oracle, and the state
    block's member order kept (every member differs from its neighbour)."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, range(100, 164))
    avg = pa.Avg(8, 3600.0)
    kw = dict(backward=pa.PA_BACKWARD_CLENSHAW, solver=pa.PA_SOLVER_CHEBYSHEV, weight_cut=0.0)
    if precision == "fp64":
        cfg = pa.solve_cfg(**kw, **PARITY)
        tol = TOL
    else:
        cfg = pa.solve_cfg(**kw, precision=pa.PA_FP32_REFINED, cheb_tol=1e-13, cg_rtol=1e-12)
        tol = 1e-10
    out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
    if precision == "fp32_refined":
        assert st["refinements"] > 0
    got = mm.back(out.cpu().numpy())
    assert np.all(np.isfinite(got))
    for m in (0, 21, 42, 63):
        ref = oo.phase_avg_rhs(lb, *onodes(avg), U[m], tol=1e-13, rtol=1e-14)
        check_parity(oo, got[m], ref, tol)
        assert rel_w(oo, got[m + 1 if m < 63 else m - 1], ref) > 1e-3


@pytest.mark.parametrize("solver", [0, 1])
def test_gpu_rest_states(solver):
    """Degenerate states.  The zero state: the averaged right-hand side, the
    nonlinearity, the step and the exponential all return exact zeros (no
    0/0 in the relative residual checks of zero right-hand sides).  A lake at
    rest (u = 0, constant depth, no topography): the discrete gradient of a
    constant and the divergence of zero flux vanish exactly, so every
    Chebyshev basis vector is +-U or 0 and N of each is exactly zero; the
    exponential and the step return U up to the Chebyshev truncation.
    t = 0: the exponential returns U."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(solver=solver, weight_cut=0.0, **PARITY)
    zero = to_dev(np.zeros((2, lo.n)))
    for out in (lo.phase_avg_rhs(avg, zero, cfg)[0], lo.swe_nonlinear(zero, cfg)[0],
                lo.expL_apply([1800.0, -900.0], zero, cfg)[0]):
        assert np.array_equal(out.cpu().numpy(), np.zeros((2, lo.n)))
    Z = zero.clone()
    lo.step(avg, 1800.0, Z, cfg)
    assert np.array_equal(Z.cpu().numpy(), np.zeros((2, lo.n)))
    rest = np.zeros((2, lo.n))
    rest[0, lm.ne:] = 7.5
    rest[1, lm.ne:] = -3.0
    R = to_dev(rest)
    nb, _ = lo.phase_avg_rhs(avg, R, cfg)
    assert np.array_equal(nb.cpu().numpy(), np.zeros((2, lo.n)))
    e, _ = lo.expL_apply([3600.0, -1800.0], R, cfg)
    assert np.abs(e.cpu().numpy() - rest).max() <= 1e-12 * 7.5
    e0, _ = lo.expL_apply(0.0, to_dev(mm.state(bumps(om, [1, 2]))), cfg)
    U = mm.state(bumps(om, [1, 2]))
    assert np.abs(e0.cpu().numpy() - U).max() <= 1e-14 * np.abs(U).max()
    lo.step(avg, 1800.0, R, cfg)
    assert np.abs(R.cpu().numpy() - rest).max() <= 1e-12 * 7.5


def test_gpu_step_parity():
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0])
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(weight_cut=0.0, **PARITY)
    Ud = to_dev(mm.state(U))
    lo.step(avg, 1800.0, Ud, cfg)
    got = mm.back(Ud.cpu().numpy())[0]
    ref = oo.step(lb, *onodes(avg), 1800.0, U[0], tol=1e-13, rtol=1e-14)
    check_parity(oo, got, ref, TOL)


def test_gpu_deterministic():
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = to_dev(mm.state(bumps(om, [0, 1])))
    avg = pa.Avg(8, 3600.0)
    a, _ = lo.phase_avg_rhs(avg, U)
    b, _ = lo.phase_avg_rhs(avg, U)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_gpu_lambda_estimate():
    om, oo, lm, lo, mm, lb = pair(3)
    est = lo.estimate_lambda(iters=200, safety=1.05)
    assert abs(est / lb - 1) < 0.03
    lo.lambda_bar = lb


def test_gpu_diagnostics_mass_energy():
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0, 1])
    d = lo.diagnostics(to_dev(mm.state(U)))
    keys = ["mass", "energy_linear", "energy_nonlinear", "hdiv_u", "l2_eta"]
    for j in range(2):
        ref = oo.diagnostics(U[j])
        for q, k in enumerate(keys):
            assert abs(d[j, q] / ref[k] - 1) < 1e-13, (k, d[j, q], ref[k])


@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 64, 65])
def test_gpu_expL_batch_shapes(B):
    """Fused (B <= 4) and finalize (B > 4) CG paths, padded column counts,
    more than one column tile (B = 65)."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(2)
    rng = np.random.default_rng(B)
    ts = rng.uniform(-5000.0, 5000.0, B)
    U = bumps(om, [j % 7 for j in range(B)])
    out, st = lo.expL_apply(ts, to_dev(mm.state(U)), pa.solve_cfg(solver=0, **PARITY))
    got = mm.back(out.cpu().numpy())
    for j in range(0, B, max(1, B // 6)):
        ref, _ = oo.expL(lb, ts[j], U[j], tol=1e-13, rtol=1e-14)
        check_parity(oo, got[j], ref, TOL)


def test_gpu_budget_mode_and_repeat():
    """Second call runs on the learned iteration budget without polling and
    gives the same result; a budget that is too small is detected and the
    call repeated with polling."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = to_dev(mm.state(bumps(om, [2])))
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(cg_rtol=1e-11, solver=0, use_graph=False)
    lo.ctx.set_cg_budget(1e-11, 0)
    a, sa = lo.phase_avg_rhs(avg, U, cfg)   # polling, learns the budget
    b, sb = lo.phase_avg_rhs(avg, U, cfg)   # budget
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert sa["budget"] == 0 and sb["budget"] > 0 and sb["fallbacks"] == 0
    lo.ctx.set_cg_budget(1e-11, 3)         # far too small: repeat with polling
    c, sc = lo.phase_avg_rhs(avg, U, cfg)
    assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())
    assert sc["fallbacks"] == 1


def test_gpu_graph_replay_matches_eager():
    """The averaged RHS captured as a HIP graph: every replay, with eager
    library work and synchronisations in between, equals the eager result;
    a different output buffer forces a new capture."""
    import torch
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = to_dev(mm.state(bumps(om, [1])))
    avg = pa.Avg(8, 3600.0)
    ref, _ = lo.phase_avg_rhs(avg, U, pa.solve_cfg(cg_rtol=1e-12, solver=0, use_graph=False))
    ref = ref.cpu().numpy()
    gcfg = pa.solve_cfg(cg_rtol=1e-12, solver=0, use_graph=True)
    out = torch.empty_like(U)
    graphs = 0
    for i in range(4):
        out.fill_(float("nan"))
        _, st = lo.phase_avg_rhs(avg, U, gcfg, out=out)
        graphs += st["graph"]
        assert np.array_equal(out.cpu().numpy(), ref), i
        lo.swe_nonlinear(U)
        torch.cuda.synchronize()
    assert graphs == 4
    out2 = torch.empty_like(U)
    _, st = lo.phase_avg_rhs(avg, U, gcfg, out=out2)
    assert st["graph"] == 1 and np.array_equal(out2.cpu().numpy(), ref)


def test_gpu_autotune_keeps_parity(tmp_path):
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0])
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(weight_cut=0.0, use_graph=True, **PARITY)
    Ud = to_dev(mm.state(U))
    cache = str(tmp_path / "tune.json")
    default = pa.get_launch_tune()
    try:
        res = lo.autotune(avg, Ud, cfg, cache=cache)
        assert res["narrow_rows_per_thread"] in (1, 2, 4, 8) and not res["cached"]
        # the choice belongs to these operators; the process default is untouched
        assert lo.has_own_tune() and pa.get_launch_tune() == default
        assert lo.get_tune() == {k: res[k] for k in pa.TUNE_FIELDS}
        lo.set_tune()
        assert not lo.has_own_tune()
        assert lo.autotune(avg, Ud, cfg, cache=cache)["cached"]
        assert lo.get_tune() == {k: res[k] for k in pa.TUNE_FIELDS}
        out, _ = lo.phase_avg_rhs(avg, Ud, cfg)
        got = mm.back(out.cpu().numpy())[0]
        ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
        check_parity(oo, got, ref, TOL)
    finally:
        lo.set_tune()


def test_gpu_launch_shapes_belong_to_operators():
    """Two operator objects with different launch shapes (CG solves, whose
    reductions group their partial sums by the grid, so the shape shows in
    the bits), run alternately and from two threads at once, each give
    exactly the result they give alone; graph replays of both keep theirs."""
    import threading
    from paper_2103_07706_amd import pa
    from gpu_common import _ctx
    om, oo, lm, lo, mm, lb = pair(4)  # 7680 rows: one and eight rows a thread differ in grid
    A = pa.Ops(_ctx(), lm)
    B = pa.Ops(_ctx(), lm)
    for o in (A, B):
        o.lambda_bar = lb
    A.set_tune(narrow_rows_per_thread=1, wide_max_wg=512)
    B.set_tune(narrow_rows_per_thread=8, wide_max_wg=2048)
    U = to_dev(mm.state(bumps(om, [3])))
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(solver=0, cg_rtol=1e-12, use_graph=False)
    a0 = A.phase_avg_rhs(avg, U, cfg)[0].cpu().numpy()
    b0 = B.phase_avg_rhs(avg, U, cfg)[0].cpu().numpy()
    assert not np.array_equal(a0, b0)  # the shapes are visible in the bits
    for _ in range(2):
        assert np.array_equal(A.phase_avg_rhs(avg, U, cfg)[0].cpu().numpy(), a0)
        assert np.array_equal(B.phase_avg_rhs(avg, U, cfg)[0].cpu().numpy(), b0)
    results = {}

    def run(name, o, ref):
        import torch
        ctx = pa.Context(0, stream=torch.cuda.Stream(0).cuda_stream)
        mine = pa.Ops(ctx, lm)
        mine.lambda_bar = lb
        mine.set_tune(**o.get_tune())
        ok = True
        for _ in range(4):
            out = mine.phase_avg_rhs(avg, U, cfg)[0]
            torch.cuda.synchronize()
            ok = ok and np.array_equal(out.cpu().numpy(), ref)
        results[name] = ok

    th = [threading.Thread(target=run, args=("A", A, a0)),
          threading.Thread(target=run, args=("B", B, b0))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert results == {"A": True, "B": True}
    gcfg = pa.solve_cfg(solver=0, cg_rtol=1e-12, use_graph=True)
    ga = A.phase_avg_rhs(avg, U, gcfg)[0].cpu().numpy()
    gb = B.phase_avg_rhs(avg, U, gcfg)[0].cpu().numpy()
    assert np.array_equal(A.phase_avg_rhs(avg, U, gcfg)[0].cpu().numpy(), ga)
    assert np.array_equal(B.phase_avg_rhs(avg, U, gcfg)[0].cpu().numpy(), gb)


def test_gpu_graph_cache_follows_object_contents():
    """A captured graph is not replayed for different averaging nodes or
    rebound operators that happen to reuse a freed object's address: each
    result equals the oracle for its own nodes."""
    import gc

    import torch
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [4])
    Ud = to_dev(mm.state(U))
    cfg = pa.solve_cfg(weight_cut=0.0, use_graph=True, **PARITY)
    out = torch.empty_like(Ud)
    for T in (3600.0, 1200.0, 3600.0, 600.0):
        avg = pa.Avg(8, T)
        _, st = lo.phase_avg_rhs(avg, Ud, cfg, out=out)
        assert st["graph"] == 1 and st["graph_captured"] == 1
        _, st = lo.phase_avg_rhs(avg, Ud, cfg, out=out)
        assert st["graph"] == 1 and st["graph_captured"] == 0
        ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
        check_parity(oo, mm.back(out.cpu().numpy())[0], ref, TOL, what=T)
        del avg
        gc.collect()
    # the operators moved to a new device buffer: the graph is captured
    # again (a replay would read the old buffer, which the caller may free)
    avg = pa.Avg(8, 3600.0)
    first = lo.phase_avg_rhs(avg, Ud, cfg, out=out)[0].cpu().numpy()
    assert lo.phase_avg_rhs(avg, Ud, cfg, out=out)[1]["graph_captured"] == 0
    lo.rebind()
    again, st = lo.phase_avg_rhs(avg, Ud, cfg, out=out)
    assert st["graph"] == 1 and st["graph_captured"] == 1
    assert np.array_equal(again.cpu().numpy(), first)


CHEB = dict(solver=1)


@pytest.mark.parametrize("backward", [0, 1])
def test_gpu_chebyshev_solver_parity(backward):
    """Reduction-free Chebyshev mass solves reach the same FP64 residual
    tolerance as CG: the averaged RHS and the exponential agree with the
    oracle (which uses CG) to the same bar."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(3)
    U = bumps(om, [0])
    avg = pa.Avg(8, 3600.0)
    cfg = pa.solve_cfg(backward=backward, weight_cut=0.0, **PARITY, **CHEB)
    out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
    # the largest final residual over all solves of the call, as checked
    assert 0 < st["resid_max"] <= PARITY["cg_rtol"]
    got = mm.back(out.cpu().numpy())[0]
    ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
    check_parity(oo, got, ref, TOL)
    ts = [900.0, -2700.0]
    U2 = bumps(om, [1, 2])
    out, _ = lo.expL_apply(ts, to_dev(mm.state(U2)), cfg)
    got = mm.back(out.cpu().numpy())
    for j, t in enumerate(ts):
        ref, _ = oo.expL(lb, t, U2[j], tol=1e-13, rtol=1e-14)
        check_parity(oo, got[j], ref, TOL)


@pytest.mark.parametrize("maxit", [3, 4])
def test_gpu_chebyshev_check_failure_falls_back(maxit):
    """Too few Chebyshev steps (maxit caps them) fail the final residual
    check; the call is repeated with CG, which then reports non-convergence
    under the same cap.  maxit 3 and 4: the single-column solves end with
    one pair of steps after a single step, or with two pairs."""
    from paper_2103_07706_amd import pa
    om, oo, lm, lo, mm, lb = pair(2)
    U = to_dev(mm.state(bumps(om, [0])))
    cfg = pa.solve_cfg(maxit=maxit, cg_rtol=1e-12, **CHEB)
    with pytest.raises(pa.PAError) as ei:
        lo.swe_nonlinear(U, cfg)
    assert ei.value.code == 4
    ok, st = lo.swe_nonlinear(U, pa.solve_cfg(cg_rtol=1e-12, **CHEB))
    assert st["fallbacks"] == 0
    ref, _ = lo.swe_nonlinear(U, pa.solve_cfg(cg_rtol=1e-12, solver=0))
    assert np.abs(ok.cpu().numpy() - ref.cpu().numpy()).max() <= 1e-9 * np.abs(ref.cpu().numpy()).max()


@pytest.mark.parametrize("backward,mixed_min_cols", [(0, 1), (1, 1), (1, 8)])
def test_gpu_fp32_refined_parity(backward, mixed_min_cols):
    """FP32 inner mass solves with FP64 residual refinement (to 1e-12):
    the averaged RHS agrees with the FP64 oracle to 1e-10 (energy norm).
    mixed_min_cols = 1: every solve refined; 8: only the 8-column solves of
    N (the single-column recurrences take FP64 steps)."""
    from paper_2103_07706_amd import pa
    keep = pa.get_launch_tune()
    pa.set_launch_tune(mixed_min_cols=mixed_min_cols)
    try:
        om, oo, lm, lo, mm, lb = pair(3)
        U = bumps(om, [0])
        avg = pa.Avg(8, 3600.0)
        cfg = pa.solve_cfg(backward=backward, weight_cut=0.0, precision=pa.PA_FP32_REFINED,
                           cheb_tol=1e-13, cg_rtol=1e-12)
        out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
        assert st["refinements"] > 0
        got = mm.back(out.cpu().numpy())[0]
        ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
        check_parity(oo, got, ref, 1e-10)
        out2, _ = lo.swe_nonlinear(to_dev(mm.state(U)), cfg)
        ref2 = oo.nonlinear(U[0], rtol=1e-14)
        check_parity(oo, mm.back(out2.cpu().numpy())[0], ref2, 1e-10)
    finally:
        pa.set_launch_tune(**keep)


@pytest.mark.parametrize("level", [2, 3, 4])
@pytest.mark.parametrize("tol", ["parity", "metric"])
def test_gpu_cheb_fused_steps(level, tol):
    """Single-column Jacobi Chebyshev solves with 2 to 6 steps per
    launch (each workgroup forms the earlier steps again on the rings of
    rows its later steps read) against one step per launch: the same Nbar
    bit for bit (every row's arithmetic is the same), residuals within the
    tolerance, and parity with the oracle.  Parts of 512 rows: a single
    ragged part at level 2, a ragged last part at level 3, whole parts at
    level 4; the step counts of the two tolerances leave
    different remainders for the first launch of a solve; the metric case
    also runs captured and replayed."""
    from paper_2103_07706_amd import pa
    keep = pa.get_launch_tune()
    try:
        om, oo, lm, lo, mm, lb = pair(level)
        U = bumps(om, [4])
        avg = pa.Avg(8, 3600.0)
        kw = PARITY if tol == "parity" else dict(cheb_tol=1e-6, cg_rtol=1e-10)
        cfg = pa.solve_cfg(backward=pa.PA_BACKWARD_CLENSHAW, weight_cut=0.0,
                           use_graph=tol == "metric", **kw, **CHEB)
        res = {}
        for fs in (1, 2, 3, 4, 5, 6):
            pa.set_launch_tune(fused_steps=fs)
            for rep in range(2 if tol == "metric" else 1):
                out, st = lo.phase_avg_rhs(avg, to_dev(mm.state(U)), cfg)
                assert 0 < st["resid_max"] <= kw["cg_rtol"], st["resid_max"]
                assert st["fallbacks"] == 0
                got = out.cpu().numpy()
                if fs in res:
                    assert np.array_equal(got, res[fs])  # graph replay
                res[fs] = got
        if tol == "parity":
            ref = oo.phase_avg_rhs(lb, *onodes(avg), U[0], tol=1e-13, rtol=1e-14)
            for fs in (1, 2, 3, 4, 5, 6):
                check_parity(oo, mm.back(res[fs])[0], ref, TOL)
        for fs in (2, 3, 4, 5, 6):
            diff = np.abs(res[fs] - res[1]).max() / np.abs(res[1]).max()
            assert np.array_equal(res[fs], res[1]), (fs, diff)
    finally:
        pa.set_launch_tune(**keep)
